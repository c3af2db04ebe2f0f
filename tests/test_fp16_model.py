"""Pins for the numpy model of the FP16 relative-coordinate test (oracle/rcll_fp16.py).

The model's rounding steps are checked against exact rational arithmetic, its stored
coordinates against the exact Eq. 6 value, its r^2 against the stated error bound,
its three-way decision against the FP64 oracle, and its neighbour count against the
oracle's. CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import rcll_fp16 as M
from paper_2401_08586_amd import workloads as W


def rn16_exact(fr: Fraction) -> float:
    """Round a rational to the nearest binary16 (ties to even), written from the format:
    10 fraction bits, exponent range [-14, 15], subnormal step 2^-24."""
    if fr == 0:
        return 0.0
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -14)
    ulp = Fraction(2) ** (e - 10)
    q, r = divmod(a, ulp)
    if r > ulp / 2 or (r == ulp / 2 and q % 2 == 1):
        q += 1
    v = q * ulp
    if v >= 65520:
        return sign * math.inf
    return sign * float(v)


def test_numpy_f16_rounding_matches_exact():
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.uniform(-8, 8, 4000), rng.uniform(-1e-4, 1e-4, 2000),
                           # exact midpoints between neighbouring f16 values
                           (np.arange(-2000, 2000) + 0.5) * 2.0 ** -10,
                           (np.arange(0, 500) + 0.5) * 2.0 ** -24])
    for v in vals:
        assert float(np.float16(v)) == rn16_exact(Fraction(float(v)))


def test_fma_emulation_is_single_rounding():
    """RN16(a*b + c) via float64 equals the exactly rounded value for f16 operands."""
    rng = np.random.default_rng(1)
    a = rng.uniform(-4, 4, 3000).astype(np.float16)
    c = rng.uniform(0, 40, 3000).astype(np.float16)
    small = (rng.uniform(-1, 1, 500) * 2.0 ** -20).astype(np.float16)      # subnormal operands
    a = np.concatenate([a, small])
    c = np.concatenate([c, rng.uniform(0, 48, 500).astype(np.float16)])
    got = (a.astype(np.float64) * a.astype(np.float64) + c.astype(np.float64)).astype(np.float16)
    for x, z, g in zip(a, c, got):
        want = rn16_exact(Fraction(float(x)) * Fraction(float(x)) + Fraction(float(z)))
        assert float(g) == want


@pytest.mark.parametrize("dim", [2, 3])
def test_stored_coordinate_error(dim):
    """|q - (2 xi - 1)| <= 2^-12 (f16) + 2^-24 (f32) + 2^(1-F) (fixed point), where xi is the
    exact position inside the cell in cell widths (Eq. 6 scale)."""
    ps = W.uniform(dim, 3000, seed=dim)
    fr = M.frame(dim, ps.lo, ps.hi, ps.cell_size, ps.radius)
    X, c, q = M.fixed_point(ps.pos, ps.lo, fr)
    w = Fraction(fr["w"])
    bound = Fraction(1, 2 ** 12) + Fraction(1, 2 ** 24) + Fraction(2, 2 ** fr["F"])
    for i in range(0, ps.n, 3):
        for k in range(dim):
            xi = (Fraction(float(ps.pos[i, k])) - Fraction(float(ps.lo[k]))) / w - int(c[i, k])
            assert abs(Fraction(float(q[i, k])) - (2 * xi - 1)) <= bound
            assert -1 <= float(q[i, k]) <= 1


def test_special_values():
    # a particle on a cell corner stores -1; coincident particles give r2 = 0
    fr = M.frame(2, (0, 0), (1, 1), 0.25, 0.25)
    p = np.array([[0.0, 0.0], [0.3, 0.7], [0.3, 0.7]])
    X, c, q = M.fixed_point(p, (0, 0), fr)
    assert float(q[0, 0]) == -1.0 and float(q[0, 1]) == -1.0
    r2, _ = M.pair_r2_16(2, q[1:2], c[1:2], q[2:3], c[2:3])
    assert float(r2[0]) == 0.0
    # thresholds bracket 4 rho^2 and lie in the f16 grid
    assert float(fr["t_lo"]) <= 4 * (fr["rho2"] - M.BAND) and float(fr["t_hi"]) >= 4 * (fr["rho2"] + M.BAND)
    assert float(fr["t_lo"]) < float(fr["t_mid"]) < float(fr["t_hi"])


@pytest.mark.parametrize("dim", [2, 3])
def test_r2_error_within_bound(dim):
    """Random pairs across adjacent cells, concentrated near the cutoff."""
    rng = np.random.default_rng(10 + dim)
    ps = W.ring_pairs(4000, 0.05, seed=dim, dim=dim, exps=(3, 5, 7, 9))
    fr = M.frame(dim, ps.lo, ps.hi, ps.cell_size, ps.radius)
    X, c, q = M.fixed_point(ps.pos, ps.lo, fr)
    i = np.arange(0, ps.n, 2)
    j = i + 1
    r2h, _ = M.pair_r2_16(dim, q[i], c[i], q[j], c[j])
    w = fr["w"]
    exact = np.array([float(sum((Fraction(float(ps.pos[b, k])) - Fraction(float(ps.pos[a, k]))) ** 2
                                for k in range(dim)) / Fraction(w) ** 2) for a, b in zip(i, j)])
    err = np.abs(r2h.astype(np.float64) / 4 - exact)
    bound = np.array([M.error_bound(dim, math.sqrt(e)) for e in exact])
    assert np.all(err <= bound)
    # the bound at the cutoff stays inside the band
    assert M.error_bound(dim, 1.0) < M.BAND
    del rng


@pytest.mark.parametrize("maker", [
    lambda: W.lattice(2, 120, 1 / 120, 0.1, seed=1),
    lambda: W.lattice(3, 24, 1 / 24, 0.1, seed=2),
    lambda: W.uniform(2, 20000, seed=3),
    lambda: W.clustered(6000, 4, dim=3),
    lambda: W.ring_pairs(3000, 0.04, seed=5, dim=3),
    lambda: W.ring_pairs(3000, 0.03, seed=6, dim=2),
], ids=["lat2d", "lat3d", "uni2d", "clu3d", "ring3d", "ring2d"])
def test_three_way_test_reproduces_oracle(maker):
    """in / band-recheck / out gives exactly the oracle's neighbour count, nothing lands
    on the wrong side of the band, and the naive FP16 errors all sit inside the band."""
    ps = maker()
    st = M.stats(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    rp, _, _ = oracle.search_ps(ps)
    assert st["misplaced"] == 0
    assert st["nnz"] == rp[-1]
    assert st["max_err_ratio"] <= 1.0
    assert st["band_pairs"] >= st["fp16_false_pos"] + st["fp16_false_neg"]


def test_candidate_count_closed_form():
    """Perfect lattice with 2 sites per cell per axis: every interior target sees 3^d cells
    of 2^d sites, minus itself."""
    n = 16
    dx = 1 / n
    ps = W.lattice(2, n, dx, jitter=0.0, radius_factor=2.0)
    # cells of width 2 dx (times the 2^-30 slack) hold exactly 2x2 sites
    st = M.stats(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    nc = st["frame"]["nc"]
    assert nc == [8, 8] or nc == [9, 9]
    # count per cell-neighbourhood directly
    cells = np.floor(ps.pos / st["frame"]["w"]).astype(int)
    tot = 0
    for a in range(ps.n):
        d = np.abs(cells - cells[a]).max(axis=1)
        tot += int((d <= 1).sum()) - 1
    assert st["candidates"] == tot
