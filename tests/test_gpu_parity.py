"""GPU parity: the HIP library through its C ABI against the CPU oracle, element by element.

Neighbour sets (row_ptr, col) must be bit-identical; FP32 distances within 1e-6 relative
(FP16 path) or bit-identical (FP64 baseline and FP32 mode, which round the same binary64
value); the
FP16 and FP32 statistics must equal the numpy models' exactly."""
import numpy as np
import pytest

import oracle
from oracle import rcll_fp16 as M
from oracle import rcll_fp32 as M32
from paper_2401_08586_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2401_08586_amd import nnps  # noqa: E402

MODES = [nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_RECHECK_ALL, nnps.MODE_FP32_RCLL]
MODE_NAMES = {0: "fp16", 1: "fp64", 2: "recheck_all", 3: "fp32"}
EXACT_DIST = (nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nnps.Context(0)
    yield c
    c.close()


def gpu_search(ctx, ps, mode):
    pos = torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda()
    cells = ctx.cells()
    rp, col, dist, _ = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, mode=mode, ctx=ctx,
                                   cells=cells)
    st = cells.stats()
    torch.cuda.synchronize()
    out = rp.cpu().numpy(), col.cpu().numpy(), dist.cpu().numpy(), st
    cells.close()
    return out


def check_against_oracle(got, want, mode, name):
    rp, col, dist, _ = got
    wrp, wcol, wdist = want
    assert rp.shape == wrp.shape, name
    np.testing.assert_array_equal(rp, wrp, err_msg=f"{name} row_ptr")
    np.testing.assert_array_equal(col, wcol, err_msg=f"{name} col")
    if mode in EXACT_DIST:
        np.testing.assert_array_equal(dist.view(np.uint32), wdist.view(np.uint32), err_msg=f"{name} dist")
    else:
        wd = wdist.astype(np.float64)
        err = np.abs(dist.astype(np.float64) - wd)
        assert np.all(err <= 1e-6 * wd), f"{name} dist max rel {np.max(err / np.maximum(wd, 1e-300))}"
        assert np.all(dist[wdist == 0] == 0)


def small_cases():
    cases = [
        W.c0(),
        W.lattice(2, 100, 0.01, 0.0, name="c0_perfect"),
        W.lattice(3, 30, 1 / 30, 0.1, seed=3, name="lat3d_30"),
        W.lattice(3, 17, 1 / 17, 0.0, name="lat3d_17_perfect"),
        W.uniform(2, 20000, seed=1),
        W.uniform(3, 20000, seed=2),
        W.clustered(8000, 5, dim=3),
        W.clustered(8000, 6, dim=2),
        W.ring_pairs(2000, 0.02, seed=7, dim=2),
        W.ring_pairs(2000, 0.05, seed=8, dim=3),
    ]
    # radius below the cell size, and a box that does not start at 0
    ps = W.uniform(3, 15000, seed=9)
    ps.cell_size = ps.radius * 1.7
    ps.name = "uniform3d_cell1.7R"
    cases.append(ps)
    ps = W.uniform(2, 15000, seed=10)
    ps.pos = ps.pos * 3.0 - 1.25
    ps.lo, ps.hi = (-1.25, -1.25), (1.75, 1.75)
    ps.radius *= 3.0
    ps.cell_size = ps.radius
    ps.name = "uniform2d_shifted"
    cases.append(ps)
    # a long thin domain: many cells along x (more than one 512-cell cut per row)
    rng = np.random.default_rng(11)
    pos = np.stack([rng.uniform(0, 40, 30000), rng.uniform(0, 0.2, 30000)], axis=1)
    cases.append(W.ParticleSet(pos, (0, 0), (40, 0.2), 0.03, 0.03, "thin2d"))
    # more than 1024 cells along z (cell indices mod 2^10 wrap inside the domain)
    pos = np.stack([rng.uniform(0, 0.1, 30000), rng.uniform(0, 0.1, 30000), rng.uniform(0, 40, 30000)], axis=1)
    cases.append(W.ParticleSet(pos, (0, 0, 0), (0.1, 0.1, 40), 0.03, 0.03, "thin3d_z"))
    return cases


@pytest.mark.parametrize("mode", MODES, ids=lambda m: MODE_NAMES[m])
@pytest.mark.parametrize("case", small_cases(), ids=lambda c: c.name)
def test_parity_small(ctx, case, mode):
    print(f"[gpu] parity {case.name} n={case.n} mode={MODE_NAMES[mode]}", flush=True)
    got = gpu_search(ctx, case, mode)
    want = oracle.search_ps(case)
    check_against_oracle(got, want, mode, case.name)
    st = got[3]
    assert st["nnz"] == want[0][-1]
    if mode == nnps.MODE_FP32_RCLL:
        # statistics of the FP32 pass (dense cells are decided in FP64 and add none)
        model = M32.stats(case.pos, case.lo, case.hi, case.cell_size, case.radius)
        if st["dense_rows"] == 0:
            assert st["candidates"] == model["candidates"]
            assert st["band_pairs"] == model["band_pairs"]
            assert st["fp16_false_pos"] == model["fp32_false_pos"]
            assert st["fp16_false_neg"] == model["fp32_false_neg"]
        else:
            assert st["band_pairs"] <= model["band_pairs"]
    elif mode != nnps.MODE_FP64_BASELINE:
        model = M.stats(case.pos, case.lo, case.hi, case.cell_size, case.radius)
        assert st["candidates"] == model["candidates"]
        assert st["band_pairs"] == model["band_pairs"]
        assert st["fp16_false_pos"] == model["fp16_false_pos"]
        assert st["fp16_false_neg"] == model["fp16_false_neg"]
        assert st["outside_band_disagree"] == 0


@pytest.mark.parametrize("which", ["c1", "c2"])
@pytest.mark.parametrize("mode", [nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL],
                         ids=lambda m: MODE_NAMES[m])
def test_parity_full_size(ctx, which, mode):
    ps = getattr(W, which)()
    print(f"[gpu] full-size parity {ps.name} n={ps.n} mode={MODE_NAMES[mode]}", flush=True)
    got = gpu_search(ctx, ps, mode)
    want = oracle.search_ps(ps)
    check_against_oracle(got, want, mode, ps.name)


def test_edge_sizes(ctx):
    for n, dim in [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (65, 2), (129, 3)]:
        rng = np.random.default_rng(n + dim)
        pos = rng.uniform(0, 1, size=(n, dim))
        ps = W.ParticleSet(pos, (0,) * dim, (1,) * dim, 0.3, 0.3, f"n{n}_{dim}d")
        print(f"[gpu] edge {ps.name}", flush=True)
        for mode in MODES:
            check_against_oracle(gpu_search(ctx, ps, mode), oracle.search_ps(ps), mode, ps.name)


def test_degenerate_inputs(ctx):
    """All particles in one cell; exact duplicates; points on cell and box faces."""
    rng = np.random.default_rng(5)
    cases = []
    pos = rng.uniform(0.4, 0.45, size=(300, 3))
    cases.append(W.ParticleSet(pos, (0, 0, 0), (1, 1, 1), 0.2, 0.2, "one_cell_3d"))
    pos = np.repeat(rng.uniform(0, 1, size=(200, 2)), 4, axis=0)
    cases.append(W.ParticleSet(pos, (0, 0), (1, 1), 0.05, 0.05, "dups_2d"))
    g = rng.integers(0, 17, size=(3000, 3)) * 0.0625
    cases.append(W.ParticleSet(g, (0, 0, 0), (1, 1, 1), 0.0625, 0.0625, "faces_3d"))
    cases.append(W.ParticleSet(g[:, :2].copy(), (0, 0), (1, 1), 0.125, 0.0625, "faces_2d"))
    for ps in cases:
        print(f"[gpu] degenerate {ps.name}", flush=True)
        for mode in MODES:
            check_against_oracle(gpu_search(ctx, ps, mode), oracle.search_ps(ps), mode, ps.name)


def test_long_rows(ctx):
    """Rows longer than the per-lane buffers take the long-row path."""
    rng = np.random.default_rng(6)
    pos = np.concatenate([rng.normal(0.5, 0.01, size=(3000, 3)), rng.uniform(0, 1, size=(3000, 3))])
    pos = np.clip(pos, 0, 1)
    ps = W.ParticleSet(pos, (0, 0, 0), (1, 1, 1), 0.05, 0.05, "long_rows_3d")
    print(f"[gpu] long rows {ps.name}", flush=True)
    want = oracle.search_ps(ps)
    ctx.set_tuning(dense_min_union=-1)  # the block and long-row paths only
    try:
        for mode in MODES:
            got = gpu_search(ctx, ps, mode)
            check_against_oracle(got, want, mode, ps.name)
            assert got[3]["heavy_rows"] > 0
    finally:
        ctx.set_tuning()
    for mode in MODES:  # default: the dense cells take the dense-cell path
        got = gpu_search(ctx, ps, mode)
        check_against_oracle(got, want, mode, ps.name + "_dense")
        assert got[3]["dense_rows"] > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_many_band_pairs_per_target(ctx, dim):
    """Centres with 24 neighbours each at distance R (1 + k 2^-12), k in {-1, 0, 1}: every
    one of them is a band pair of its centre, more than the count pass queues per target,
    so the rest are decided on the spot; the CSR and the FP16 statistics must still be
    the oracle's and the model's."""
    rng = np.random.default_rng(40 + dim)
    R = 0.02
    side = 12
    g = (np.stack(np.meshgrid(*[np.arange(side)] * dim, indexing="ij"), -1).reshape(-1, dim) + 0.5) * (3.2 * R)
    pts = [g]
    for k in (-1, 0, 1):
        for _ in range(8):
            d = rng.normal(size=g.shape)
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts.append(g + d * R * (1.0 + k * 2.0 ** -12))
    pos = np.concatenate(pts)
    box = side * 3.2 * R
    ps = W.ParticleSet(np.ascontiguousarray(pos), (0.0,) * dim, (box,) * dim, R, R, f"band_shells_{dim}d")
    print(f"[gpu] band shells {ps.name} n={ps.n}", flush=True)
    want = oracle.search_ps(ps)
    got = gpu_search(ctx, ps, nnps.MODE_FP16_RCLL)
    check_against_oracle(got, want, nnps.MODE_FP16_RCLL, ps.name)
    model = M.stats(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    st = got[3]
    assert model["band_pairs"] >= 24 * side ** dim
    for key in ("candidates", "band_pairs", "fp16_false_pos", "fp16_false_neg"):
        assert st[key] == model[key], key


@pytest.mark.parametrize("radius_factor,block_target", [(2.6, 80), (2.6, 128), (2.4, 128), (2.9, 64)])
def test_block_shape_stays_within_the_fill_limits(ctx, radius_factor, block_target):
    """More neighbours per particle than the default workloads, and large block targets:
    the host caps a block's x-span (union) and target count (entries) so blocks stay on the
    block path (no long rows), and the result is the oracle's."""
    ps = W.lattice(3, 26, 1 / 26, 0.1, seed=4, radius_factor=radius_factor,
                   name=f"lat3d_R{radius_factor}_bt{block_target}")
    print(f"[gpu] block limits {ps.name}", flush=True)
    want = oracle.search_ps(ps)
    ctx.set_tuning(block_target=block_target, dense_min_union=-1)
    try:
        got = gpu_search(ctx, ps, nnps.MODE_FP16_RCLL)
    finally:
        ctx.set_tuning()
    check_against_oracle(got, want, nnps.MODE_FP16_RCLL, ps.name)
    assert got[3]["heavy_rows"] == 0, ps.name


def test_deterministic(ctx):
    ps = W.clustered(20000, 12, dim=3)
    a = gpu_search(ctx, ps, nnps.MODE_FP16_RCLL)
    b = gpu_search(ctx, ps, nnps.MODE_FP16_RCLL)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_domain_error(ctx):
    pos = torch.tensor([[0.5, 0.5], [0.2, 1.5]], dtype=torch.float64, device="cuda")
    with pytest.raises(nnps.NnpsError) as e:
        nnps.search(pos, (0, 0), (1, 1), 0.1, 0.1, ctx=ctx)
    assert e.value.code == nnps.NNPS_EDOMAIN
    pos = torch.tensor([[0.5, float("nan")]], dtype=torch.float64, device="cuda")
    with pytest.raises(nnps.NnpsError) as e:
        nnps.search(pos, (0, 0), (1, 1), 0.1, 0.1, ctx=ctx)
    assert e.value.code == nnps.NNPS_EDOMAIN


def test_capacity_error(ctx):
    ps = W.c0()
    pos = torch.from_numpy(ps.pos).cuda()
    cells = ctx.cells()
    cells.build(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    rp = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
    nnz = cells.count(rp)
    col = torch.empty(nnz - 5, dtype=torch.int32, device="cuda")
    dist = torch.empty(nnz - 5, dtype=torch.float32, device="cuda")
    cells.fill(rp, col, dist)
    with pytest.raises(nnps.NnpsError) as e:
        cells.stats()
    assert e.value.code == nnps.NNPS_ECAPACITY
    cells.close()
