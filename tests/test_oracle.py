"""Pins for the CPU oracle: hand-enumerated cases, the all-list brute force, closed-form
lattice counts, symmetry and equivariance, and a library k-d tree. CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2401_08586_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rows_of(rp, col, dist):
    return [(col[rp[i]:rp[i + 1]], dist[rp[i]:rp[i + 1]]) for i in range(len(rp) - 1)]


def assert_same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# --- hand-enumerated cases (tests/golden/hand_cases.json) -----------------------------
@pytest.mark.parametrize("brute", [False, True])
def test_hand_cases(brute):
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        pos = np.array(c["pos"], dtype=np.float64)
        rp, col, dist = oracle.search(pos, c["lo"], c["hi"], c["cell_size"], c["radius"], brute=brute)
        got = rows_of(rp, col, dist)
        assert len(got) == len(c["rows"]), c["name"]
        for (gc, gd), want in zip(got, c["rows"]):
            assert list(gc) == [j for j, _ in want], c["name"]
            for d, (_, wd) in zip(gd, want):
                assert abs(float(d) - wd) <= 1e-6 * wd, (c["name"], d, wd)


# --- brute force (all-list) vs cell link list -----------------------------------------
def _random_cases():
    rng = np.random.default_rng(1234)
    cases = []
    for dim in (2, 3):
        for n in (0, 1, 2, 7, 60, 700, 2500):
            lo = rng.uniform(-3, 1, size=dim)
            span = rng.uniform(0.5, 4, size=dim)
            hi = lo + span
            cell = float(rng.uniform(0.03, 0.4)) * float(span.min())
            radius = cell * float(rng.choice([1.0, 0.999, 0.6, 0.25]))
            pos = lo + rng.uniform(0, 1, size=(n, dim)) * span
            cases.append((f"uniform{dim}d_{n}", pos, lo, hi, cell, radius))
    # duplicates and points exactly on cell faces and on the box faces
    for dim in (2, 3):
        lo = np.zeros(dim)
        hi = np.ones(dim)
        cell = 0.125
        g = rng.integers(0, 9, size=(400, dim)) * cell          # on cell faces, incl. 0 and 1
        dup = np.repeat(rng.uniform(0, 1, size=(50, dim)), 3, axis=0)
        pos = np.concatenate([g, dup, np.clip(g + 1e-17, 0, 1)])
        cases.append((f"faces{dim}d", pos, lo, hi, cell, cell))
        cases.append((f"faces{dim}d_r06", pos, lo, hi, cell, 0.6 * cell))
    # clustered and a near-cutoff ring
    ps = W.clustered(3000, 7, dim=3)
    cases.append(("clustered3d", ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius))
    ps = W.clustered(3000, 8, dim=2)
    cases.append(("clustered2d", ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius))
    for dim in (2, 3):
        ps = W.ring_pairs(300, 0.05, seed=dim, dim=dim)
        cases.append((f"ring{dim}d", ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius))
    return cases


@pytest.mark.parametrize("case", _random_cases(), ids=lambda c: c[0])
def test_cell_list_equals_brute_force(case):
    name, pos, lo, hi, cell, radius = case
    a = oracle.search(pos, lo, hi, cell, radius)
    b = oracle.search(pos, lo, hi, cell, radius, brute=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# --- closed forms on perfect lattices --------------------------------------------------
def lattice_nnz(n, dim, ratio2):
    """sum over offsets o != 0 with |o|^2 <= ratio2 of prod_k (n - |o_k|)."""
    m = int(math.isqrt(int(ratio2))) + 1
    tot = 0
    for o in itertools.product(range(-m, m + 1), repeat=dim):
        s = sum(v * v for v in o)
        if s == 0 or s > ratio2:
            continue
        tot += math.prod(max(n - abs(v), 0) for v in o)
    return tot


def test_closed_form_formula_values():
    # interior counts and totals for radius 2.4 dx (h = 1.2 dx, radius 2h)
    assert lattice_nnz(100, 2, 5.76) == 195_620
    assert lattice_nnz(1000, 2, 5.76) == 19_956_020
    assert lattice_nnz(100, 3, 5.76) == 54_628_392


@pytest.mark.parametrize("dim,n", [(2, 100), (2, 37), (3, 30), (3, 11), (2, 1000), (3, 100)])
def test_perfect_lattice_counts(dim, n):
    ps = W.lattice(dim, n, 1.0 / n, jitter=0.0)
    rp, col, dist = oracle.search_ps(ps)
    assert rp[-1] == lattice_nnz(n, dim, 5.76)
    counts = np.diff(rp)
    if n >= 5:
        # a particle with two full lattice layers on every side
        idx = 2 + n * 2 + (n * n * 2 if dim == 3 else 0)
        assert counts[idx] == (20 if dim == 2 else 56)


@pytest.mark.parametrize("dim", [2, 3])
def test_perfect_lattice_distances(dim):
    n = 12
    dx = 1.0 / n
    ps = W.lattice(dim, n, dx, jitter=0.0)
    rp, col, dist = oracle.search_ps(ps)
    site = np.stack(np.unravel_index(np.arange(n ** dim), (n,) * dim)[::-1], axis=1)
    rows = np.repeat(np.arange(n ** dim), np.diff(rp))
    m = np.sum((site[col] - site[rows]) ** 2, axis=1)
    want = dx * np.sqrt(m)
    assert np.all(np.abs(dist - want) <= 1e-6 * want)
    assert set(np.unique(m)) <= {1, 2, 4, 5} | ({3} if dim == 3 else set())


# --- invariants ------------------------------------------------------------------------
@pytest.fixture(scope="module")
def jittered():
    return [W.lattice(2, 60, 1 / 60, 0.1, seed=5), W.lattice(3, 20, 1 / 20, 0.1, seed=6),
            W.clustered(4000, 9, dim=3)]


def test_symmetry(jittered):
    for ps in jittered:
        rp, col, dist = oracle.search_ps(ps)
        rows = np.repeat(np.arange(ps.n), np.diff(rp))
        fwd = {(int(i), int(j)): d for i, j, d in zip(rows, col, dist.view(np.uint32))}
        for (i, j), d in fwd.items():
            assert fwd[(j, i)] == d


def test_permutation_equivariance(jittered):
    rng = np.random.default_rng(0)
    for ps in jittered:
        rp, col, dist = oracle.search_ps(ps)
        perm = rng.permutation(ps.n)          # new index k holds old particle perm[k]
        inv = np.argsort(perm)
        rp2, col2, dist2 = oracle.search(ps.pos[perm], ps.lo, ps.hi, ps.cell_size, ps.radius)
        for k in range(0, ps.n, 7):
            old = perm[k]
            a = dict(zip(col[rp[old]:rp[old + 1]], dist[rp[old]:rp[old + 1]]))
            b = {int(perm[j]): d for j, d in zip(col2[rp2[k]:rp2[k + 1]], dist2[rp2[k]:rp2[k + 1]])}
            assert a == b
        assert np.all(np.diff(col2)[np.diff(np.repeat(np.arange(ps.n), np.diff(rp2))) == 0] > 0)
        del inv


@pytest.mark.parametrize("k", [-3, 5])
def test_power_of_two_scaling(jittered, k):
    s = 2.0 ** k
    for ps in jittered:
        a = oracle.search_ps(ps)
        b = oracle.search(ps.pos * s, tuple(np.multiply(ps.lo, s)), tuple(np.multiply(ps.hi, s)),
                          ps.cell_size * s, ps.radius * s)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_array_equal(a[2] * np.float32(s), b[2])


def test_axis_swap(jittered):
    for ps in jittered:
        a = oracle.search_ps(ps)
        p = ps.pos.copy()
        p[:, [0, 1]] = p[:, [1, 0]]
        lo = list(ps.lo)
        hi = list(ps.hi)
        lo[0], lo[1] = lo[1], lo[0]
        hi[0], hi[1] = hi[1], hi[0]
        b = oracle.search(p, lo, hi, ps.cell_size, ps.radius)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


# --- an independent library: scipy's k-d tree -------------------------------------------
def test_kdtree_cross_check(jittered):
    from scipy.spatial import cKDTree
    for ps in jittered + [W.uniform(3, 5000, seed=3), W.uniform(2, 8000, seed=4)]:
        rp, col, dist = oracle.search_ps(ps)
        rows = np.repeat(np.arange(ps.n), np.diff(rp))
        mine = {(int(i), int(j)) for i, j in zip(rows, col) if i < j}
        tree = cKDTree(ps.pos)
        ref = tree.query_pairs(ps.radius, output_type="set")
        # the two agree away from exact ties; show no pair sits within 1e-12 of the cutoff
        diff = mine ^ ref
        assert not diff
        allp = np.array(sorted(tree.query_pairs(ps.radius * 1.01)))
        if len(allp):
            d2 = np.sum((ps.pos[allp[:, 0]] - ps.pos[allp[:, 1]]) ** 2, axis=1)
            assert np.min(np.abs(d2 - ps.radius ** 2)) / ps.radius ** 2 > 1e-12


def test_rows_subset_matches_full(jittered):
    ps = jittered[2]
    rp, col, dist = oracle.search_ps(ps)
    rows = np.array([5, 0, ps.n - 1, 17, 5])
    rp2, col2, dist2 = oracle.search_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows)
    for k, r in enumerate(rows):
        np.testing.assert_array_equal(col2[rp2[k]:rp2[k + 1]], col[rp[r]:rp[r + 1]])
        np.testing.assert_array_equal(dist2[rp2[k]:rp2[k + 1]], dist[rp[r]:rp[r + 1]])


# --- validation -------------------------------------------------------------------------
def test_validation_errors():
    p = np.array([[0.5, 0.5], [0.2, 0.3]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.search(p, (0, 0), (1, 1), 0.1, 0.2)          # radius > cell
    assert e.value.code == oracle.ORC_EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.search(p, (0, 0), (0, 1), 0.2, 0.2)          # empty box
    assert e.value.code == oracle.ORC_EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.search(np.array([[0.5, 1.5]]), (0, 0), (1, 1), 0.2, 0.2)
    assert e.value.code == oracle.ORC_EDOMAIN
    with pytest.raises(oracle.OracleError) as e:
        oracle.search(np.array([[0.5, np.nan]]), (0, 0), (1, 1), 0.2, 0.2)
    assert e.value.code == oracle.ORC_EDOMAIN
    rp, col, dist = oracle.search(np.zeros((0, 3)), (0, 0, 0), (1, 1, 1), 0.2, 0.2)
    assert list(rp) == [0] and col.size == 0


# --- the row-parallel forms (count_rows, search_par) ----------------------------------
@pytest.mark.parametrize("case", _random_cases()[::3], ids=lambda c: c[0])
@pytest.mark.parametrize("threads", [1, 4])
def test_parallel_forms_equal_brute_force(case, threads):
    """Rows computed in parallel give the brute force's CSR, and the row counts its row
    lengths, whatever the thread count."""
    name, pos, lo, hi, cell, radius = case
    want = oracle.search(pos, lo, hi, cell, radius, brute=True)
    got = oracle.search_par(pos, lo, hi, cell, radius, threads=threads)
    for x, y in zip(got, want):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(oracle.count_rows(pos, lo, hi, cell, radius, threads=threads),
                                  np.diff(want[0]))


@pytest.mark.parametrize("dim,n", [(2, 100), (3, 30), (2, 1000)])
def test_parallel_forms_perfect_lattice_totals(dim, n):
    ps = W.lattice(dim, n, 1.0 / n, jitter=0.0)
    counts = oracle.count_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, threads=4)
    assert counts.sum() == lattice_nnz(n, dim, 5.76)
    assert counts.max() == (20 if dim == 2 else 56)


def test_parallel_forms_selected_rows():
    ps = W.clustered(5000, 9, dim=3)
    rows = np.random.default_rng(1).choice(ps.n, 300, replace=False)
    want = oracle.search_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows)
    got = oracle.search_par(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows=rows, threads=3)
    for x, y in zip(got, want):
        np.testing.assert_array_equal(x, y)
    cnt = oracle.count_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows=rows, threads=2)
    np.testing.assert_array_equal(cnt, np.diff(want[0]))
    with pytest.raises(oracle.OracleError):
        oracle.count_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows=np.array([ps.n]))
    bad = ps.pos.copy()
    bad[3, 0] = 1.5
    with pytest.raises(oracle.OracleError):
        oracle.search_par(bad, ps.lo, ps.hi, ps.cell_size, ps.radius)
