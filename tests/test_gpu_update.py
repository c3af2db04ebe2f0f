"""GPU parity of the incremental update (nnps_cells_update, nnps_batch_update_step): after
several steps of moves that change the cells of most particles (and push some onto the box
faces), the count and fill on the updated structure must give exactly what a fresh build
on the moved positions gives (row_ptr, col and dist bit for bit, the same FP16
statistics), and the CPU oracle's lists on the moved binary64 positions."""
import numpy as np
import pytest

import oracle
from paper_2401_08586_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2401_08586_amd import nnps  # noqa: E402

MODES = [nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL]
MODE_IDS = ["fp16", "fp64", "fp32"]
# heavy_rows is left out: which rows of a large cell go to the long-row path depends on how
# the cell's particles fall into work blocks, i.e. on their order inside the cell
STAT_KEYS = ("nnz", "candidates", "band_pairs", "fp16_false_pos", "fp16_false_neg", "dense_rows")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nnps.Context(0)
    yield c
    c.close()


def count_fill(cells, n, dev="cuda"):
    rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nnz = cells.count(rp)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    dist = torch.empty(nnz, dtype=torch.float32, device=dev)
    cells.fill(rp, col, dist)
    return rp, col, dist


def check_oracle(got, pos, ps, name):
    rp, col, dist = (t.cpu().numpy() for t in got)
    wrp, wcol, wdist = oracle.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    np.testing.assert_array_equal(rp, wrp, err_msg=f"{name} row_ptr")
    np.testing.assert_array_equal(col, wcol, err_msg=f"{name} col")
    wd = wdist.astype(np.float64)
    assert np.all(np.abs(dist - wd) <= 1e-6 * wd), name


def check_same(a, b, name):
    for x, y, what in zip(a, b, ("row_ptr", "col", "dist")):
        xa, ya = x.cpu().numpy(), y.cpu().numpy()
        assert xa.shape == ya.shape, f"{name} {what} shape"
        assert np.array_equal(xa.view(np.uint8), ya.view(np.uint8)), f"{name} {what} differs"


def rebuilt(ctx, pos_gpu, ps, mode):
    """A fresh build + count + fill on a copy of the positions."""
    p = pos_gpu.clone()
    c = ctx.cells()
    c.build(p, ps.lo, ps.hi, ps.cell_size, ps.radius, mode)
    got = count_fill(c, ps.n)
    st = c.stats()
    c.close()
    return got, st


def workloads(dim):
    if dim == 2:
        return [W.lattice(2, 70, 1 / 70, 0.1, seed=5), W.clustered(6000, 11, dim=2), W.uniform(2, 4000, seed=3)]
    return [W.lattice(3, 18, 1 / 18, 0.1, seed=6), W.clustered(8000, 12, dim=3), W.uniform(3, 5000, seed=4)]


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("dim", [2, 3])
def test_update_matches_rebuild_and_oracle(ctx, dim, mode):
    for ps in workloads(dim):
        print(f"[gpu] update dim={dim} mode={mode} {ps.name} n={ps.n}", flush=True)
        pos = torch.from_numpy(ps.pos.copy()).cuda()
        host = ps.pos.copy()
        cells = ctx.cells()
        cells.build(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, mode)
        count_fill(cells, ps.n)
        moved_total = 0
        for step in range(4):
            # a third of a cell width per component: most particles change cell over the steps
            d = W.reflected_displacement(host, ps.lo, ps.hi, 0.3 * ps.cell_size, seed=[dim, mode, step])
            cells.update(torch.from_numpy(d).cuda())
            got = count_fill(cells, ps.n)
            st = cells.stats()
            new = host + d
            moved_total += int(np.any(np.floor(new / ps.cell_size) != np.floor(host / ps.cell_size), axis=1).sum())
            host = new
            # the library advanced the caller's positions in place, one binary64 addition each
            assert np.array_equal(pos.cpu().numpy().view(np.uint64), host.view(np.uint64)), f"{ps.name} positions"
            ref, rst = rebuilt(ctx, pos, ps, mode)
            check_same(got, ref, f"{ps.name} step {step}")
            for k in STAT_KEYS:
                assert st[k] == rst[k], (ps.name, step, k, st[k], rst[k])
            check_oracle(got, host, ps, f"{ps.name} step {step}")
        assert moved_total > ps.n // 2, f"{ps.name}: too few cell changes ({moved_total}) to test migration"
        cells.close()


def test_update_in_place_moves_and_box_faces(ctx):
    """The caller moves the positions itself (no displacement array), some onto the box
    faces and corners exactly, some across several cells at once."""
    ps = W.clustered(5000, 21, dim=3)
    rng = np.random.default_rng(7)
    pos = torch.from_numpy(ps.pos.copy()).cuda()
    cells = ctx.cells()
    cells.build(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    count_fill(cells, ps.n)
    host = ps.pos.copy()
    for step in range(3):
        host = host + rng.uniform(-0.02, 0.02, size=host.shape)
        host = np.clip(host, 0.0, 1.0)
        idx = rng.choice(ps.n, size=200, replace=False)
        host[idx[:70], 0] = 0.0
        host[idx[70:140], 1] = 1.0
        host[idx[140:], :] = rng.choice([0.0, 1.0], size=(60, 3))  # corners
        jump = rng.choice(ps.n, size=100, replace=False)
        host[jump] = rng.uniform(0, 1, size=(100, 3))  # far moves
        pos.copy_(torch.from_numpy(host))
        print(f"[gpu] update in place step {step}", flush=True)
        cells.update(None)
        got = count_fill(cells, ps.n)
        ref, _ = rebuilt(ctx, pos, ps, nnps.MODE_FP16_RCLL)
        check_same(got, ref, f"in place step {step}")
        check_oracle(got, host, ps, f"in place step {step}")
    cells.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_update_dense_cells_and_half_lists(ctx, dim):
    """Every cell through the dense-cell path, then half lists, on updated structures."""
    ps = W.clustered(7000, 31 + dim, dim=dim)
    for dense, half in ((1, False), (0, True), (1, True)):
        ctx.set_tuning(dense_min_union=dense)
        try:
            pos = torch.from_numpy(ps.pos.copy()).cuda()
            host = ps.pos.copy()
            cells = ctx.cells()
            cells.set_half(half)
            cells.build(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
            count_fill(cells, ps.n)
            for step in range(2):
                d = W.reflected_displacement(host, ps.lo, ps.hi, 0.4 * ps.cell_size, seed=[dim, step, 9])
                print(f"[gpu] update dense={dense} half={half} dim={dim} step {step}", flush=True)
                cells.update(torch.from_numpy(d).cuda())
                host = host + d
                got = count_fill(cells, ps.n)
                st = cells.stats()
                if dense:
                    assert st["dense_rows"] > 0
                c2 = ctx.cells()
                c2.set_half(half)
                c2.build(pos.clone(), ps.lo, ps.hi, ps.cell_size, ps.radius)
                ref = count_fill(c2, ps.n)
                c2.close()
                check_same(got, ref, f"dense={dense} half={half} step {step}")
                if not half:
                    check_oracle(got, host, ps, f"dense={dense} step {step}")
            cells.close()
        finally:
            ctx.set_tuning()


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graph"])
def test_batch_update_step(ctx, graphs):
    """Uneven batch (an empty set included), displacements for some sets and none for
    others, replayed as one captured update + count + fill per step."""
    pss = [W.clustered(3000, 41, dim=3), W.ParticleSet(np.zeros((0, 3)), (0, 0, 0), (1, 1, 1), 0.1, 0.1, "empty"),
           W.lattice(3, 16, 1 / 16, 0.1, seed=8), W.uniform(3, 6000, seed=9)]
    pos = [torch.from_numpy(ps.pos.copy()).cuda() for ps in pss]
    host = [ps.pos.copy() for ps in pss]
    sets = [(p, ps.lo, ps.hi, ps.cell_size, ps.radius) for p, ps in zip(pos, pss)]
    cells = ctx.cells()
    cells.set_graphs(graphs)
    res, _ = nnps.search_batch(sets, ctx=ctx)
    caps = [int(r[1].numel() * 1.5) + 1024 for r in res]
    rps = [torch.empty(ps.n + 1, dtype=torch.int64, device="cuda") for ps in pss]
    cols = [torch.empty(k, dtype=torch.int32, device="cuda") for k in caps]
    dists = [torch.empty(k, dtype=torch.float32, device="cuda") for k in caps]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cells.batch_step(sets, rps, cols, dists, stream=stream)
        for step in range(5):
            disp = []
            for s, ps in enumerate(pss):
                if ps.n == 0 or (step + s) % 3 == 2:
                    disp.append(None)  # this set does not move this step
                    continue
                d = W.reflected_displacement(host[s], ps.lo, ps.hi, 0.3 * ps.cell_size, seed=[s, step, 77])
                host[s] = host[s] + d
                disp.append(torch.from_numpy(d).cuda())
            print(f"[gpu] batch update step {step} graphs={graphs}", flush=True)
            cells.batch_update_step(rps, cols, dists, disp=disp, stream=stream)
            nnz = cells.batch_nnz(stream=stream)
            stream.synchronize()
            for s, ps in enumerate(pss):
                k = nnz[s]
                assert np.array_equal(pos[s].cpu().numpy().view(np.uint64), host[s].view(np.uint64))
                check_oracle((rps[s], cols[s][:k], dists[s][:k]), host[s], ps, f"{ps.name} step {step}")
    cells.close()


def test_update_reflects_at_box_faces(ctx):
    """Raw displacements (not pre-reflected) pushing particles through every box face: a
    component whose sum leaves the box moves by -d instead, exactly as numpy's binary64
    arithmetic gives it, and the lists match the oracle on the reflected positions."""
    rng = np.random.default_rng(17)
    for dim in (2, 3):
        ps = W.uniform(dim, 6000, seed=40 + dim)
        lo, hi = np.asarray(ps.lo), np.asarray(ps.hi)
        pos = torch.from_numpy(ps.pos.copy()).cuda()
        host = ps.pos.copy()
        cells = ctx.cells()
        cells.build(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
        count_fill(cells, ps.n)
        for step in range(3):
            d = rng.uniform(-0.5, 0.5, size=host.shape) * ps.cell_size
            print(f"[gpu] update reflect dim={dim} step {step}", flush=True)
            q = host + d
            want = np.where((q >= lo) & (q <= hi), q, host - d)
            assert np.any((q < lo) | (q > hi)), "no component crosses a face"
            cells.update(torch.from_numpy(d).cuda())
            assert np.array_equal(pos.cpu().numpy().view(np.uint64), want.view(np.uint64)), f"dim {dim} step {step}"
            host = want
            got = count_fill(cells, ps.n)
            check_oracle(got, host, ps, f"reflect dim {dim} step {step}")
        cells.close()


def test_update_errors(ctx):
    cells = ctx.cells()
    with pytest.raises(nnps.NnpsError) as e:
        cells.update(None)
    assert e.value.code == nnps.NNPS_EORDER
    ps = W.uniform(3, 2000, seed=12)
    pos = torch.from_numpy(ps.pos.copy()).cuda()
    cells.build(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    count_fill(cells, ps.n)
    d = np.zeros_like(ps.pos)
    d[17, 1] = 2.0  # leaves the box
    print("[gpu] update out of the box", flush=True)
    cells.update(torch.from_numpy(d).cuda())
    rp = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(nnps.NnpsError) as e:
        cells.count(rp)
    assert e.value.code == nnps.NNPS_EDOMAIN
    # moved back inside, the next update is clean again
    d[17, 1] = -2.0
    cells.update(torch.from_numpy(d).cuda())
    got = count_fill(cells, ps.n)
    check_oracle(got, pos.cpu().numpy(), ps, "after domain error")
    cells.close()
