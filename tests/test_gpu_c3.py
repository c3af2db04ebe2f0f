"""The clustered 32-set batch at full size (5.6 million particles, about 1e10 pairs; sizes
log-uniform in [1e4, 1e6]) against the oracle:

* every row length of every set, exactly: the SHA-256 of each set's row lengths against the
  one tests/golden/make_c3_rowcounts.py stored from the oracle's row counts (and each
  set's total); the smaller sets are also counted by the oracle here and compared row by
  row;
* at least 1 % of the rows of every set (random rows plus the longest ones), element by
  element: columns equal, distances within 1e-6 relative;
* the whole CSR on the device: every row strictly ascending, every column a set-local
  index."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2401_08586_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2401_08586_amd import nnps  # noqa: E402

CHUNK = 1 << 28
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_rowcounts.json")
LIVE_COUNT_MAX_N = 60000  # sets up to this size are also counted by the oracle in the test


def digest(counts):
    return hashlib.sha256(np.ascontiguousarray(counts, dtype="<i8").tobytes()).hexdigest()


def gather_rows(rp, t, rows, rpc):
    """Concatenated entries of the listed rows of a device CSR array, on the host."""
    starts = torch.from_numpy(rpc[rows]).cuda()
    lens = torch.from_numpy(rpc[rows + 1] - rpc[rows]).cuda()
    base = torch.repeat_interleave(starts - torch.cumsum(lens, 0) + lens, lens)
    idx = base + torch.arange(int(lens.sum()), device="cuda", dtype=torch.int64)
    return t[idx].cpu().numpy()


def test_clustered_batch_full_row_counts_and_sampled_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open(GOLDEN) as f:
        gold = json.load(f)["sets"]
    pss = W.clustered_batch()
    assert [g["n"] for g in gold] == [p.n for p in pss]
    print(f"[gpu] clustered batch: {len(pss)} sets, {sum(p.n for p in pss)} particles", flush=True)
    ctx = nnps.Context(0)
    cells = ctx.cells()
    sets = [(torch.from_numpy(p.pos).cuda(), p.lo, p.hi, p.cell_size, p.radius) for p in pss]
    res, _ = nnps.search_batch(sets, ctx=ctx, cells=cells)
    st = cells.stats()
    print(f"[gpu] nnz={st['nnz']} heavy_rows={st['heavy_rows']} dense_rows={st['dense_rows']} "
          f"band={st['band_pairs']}", flush=True)
    assert st["nnz"] == sum(int(r[1].numel()) for r in res) == sum(g["nnz"] for g in gold)
    rng = np.random.default_rng(11)
    sampled = 0
    for s, (ps, (rp, col, dist), g) in enumerate(zip(pss, res, gold)):
        rpc = rp.cpu().numpy()
        lens = np.diff(rpc)
        assert int(rpc[-1]) == g["nnz"], f"set {s} nnz"
        assert digest(lens) == g["counts_sha256"], f"set {s}: row lengths differ from the oracle's"
        if ps.n <= LIVE_COUNT_MAX_N:
            want = oracle.count_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
            np.testing.assert_array_equal(lens, want, err_msg=f"set {s} row lengths")
        k = max(40, -(-ps.n // 100))
        rows = np.unique(np.concatenate([rng.choice(ps.n, size=min(k, ps.n), replace=False),
                                         np.argsort(lens, kind="stable")[-3:]]))
        wrp, wcol, wdist = oracle.search_par(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows=rows)
        np.testing.assert_array_equal(lens[rows], np.diff(wrp), err_msg=f"set {s} sampled row lengths")
        gcol = gather_rows(rp, col, rows, rpc)
        gdist = gather_rows(rp, dist, rows, rpc).astype(np.float64)
        np.testing.assert_array_equal(gcol, wcol, err_msg=f"set {s} sampled rows")
        wd = wdist.astype(np.float64)
        assert np.all(np.abs(gdist - wd) <= 1e-6 * wd), f"set {s} distances"
        sampled += rows.size
        # whole CSR, on the device: columns in range, rows strictly ascending
        assert int(col.min()) >= 0 and int(col.max()) < ps.n, s
        down = []
        for i0 in range(1, col.numel(), CHUNK):  # torch.nonzero is kept under 2^31 elements
            i1 = min(i0 + CHUNK, col.numel())
            down.append(torch.nonzero(col[i0:i1] <= col[i0 - 1:i1 - 1]).flatten().cpu().numpy() + i0)
        down = np.concatenate(down) if down else np.zeros(0, np.int64)
        starts = set(rpc[1:-1][lens[1:] > 0].tolist())
        assert all(int(i) in starts for i in down), f"set {s}: a row is not ascending"
        assert bool((dist >= 0).all())
        print(f"[gpu] set {s} n={ps.n} nnz={g['nnz']} rows ok ({rows.size} sampled)", flush=True)
    assert sampled >= sum(p.n for p in pss) // 100
    del res
    cells.close()
    ctx.close()
    torch.cuda.empty_cache()
