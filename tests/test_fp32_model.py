"""Pins for the numpy model of the FP32 relative-coordinate test (oracle/rcll_fp32.py).

Its float32 steps are checked against exact rational rounding, its stored coordinates
against the exact Eq. 6 value, its r^2 against the stated bound (exact rationals), its
three-way decision against the FP64 oracle, and its accuracy against the FP16 model's.
CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import rcll_fp16 as M16
from oracle import rcll_fp32 as M
from paper_2401_08586_amd import workloads as W


def rn32_exact(fr: Fraction) -> float:
    """Round a rational to the nearest binary32 (ties to even), written from the format:
    23 fraction bits, exponent range [-126, 127] (no overflow or subnormals reached here)."""
    if fr == 0:
        return 0.0
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    assert -126 <= e <= 127
    ulp = Fraction(2) ** (e - 23)
    q, r = divmod(a, ulp)
    if r > ulp / 2 or (r == ulp / 2 and q % 2 == 1):
        q += 1
    return sign * float(q * ulp)


def test_numpy_f32_operations_round_exactly():
    rng = np.random.default_rng(0)
    a = rng.uniform(-4, 4, 3000).astype(np.float32)
    b = rng.uniform(-4, 4, 3000).astype(np.float32)
    # operands one ulp apart and exact midpoints of products
    b[:300] = np.nextafter(a[:300], np.float32(9))
    for x, y in zip(a, b):
        fx, fy = Fraction(float(x)), Fraction(float(y))
        assert float(x - y) == rn32_exact(fx - fy)
        assert float(x + y) == rn32_exact(fx + fy)
        assert float(x * x) == rn32_exact(fx * fx)
    d = np.array([3, 2 ** 24 + 1, 2 ** 25 + 3, -(2 ** 30) - 7, 2 ** 39 - 1], dtype=np.int64)
    for v in d:
        assert float(np.int64(v).astype(np.float32)) == rn32_exact(Fraction(int(v)))


@pytest.mark.parametrize("dim", [2, 3])
def test_stored_coordinate_error(dim):
    """|q - (2 xi - 1)| <= 2^-25 (f32) + 2^(1-F) (fixed point), xi the exact position inside
    the cell in cell widths (Eq. 6 scale)."""
    ps = W.uniform(dim, 3000, seed=dim)
    fr = M.frame(dim, ps.lo, ps.hi, ps.cell_size, ps.radius)
    X, c, q = M.fixed_point(ps.pos, ps.lo, fr)
    assert q.dtype == np.float32
    w = Fraction(fr["w"])
    bound = Fraction(1, 2 ** 25) + Fraction(2, 2 ** fr["F"])
    for i in range(0, ps.n, 3):
        for k in range(dim):
            xi = (Fraction(float(ps.pos[i, k])) - Fraction(float(ps.lo[k]))) / w - int(c[i, k])
            assert abs(Fraction(float(q[i, k])) - (2 * xi - 1)) <= bound
            assert -1 <= float(q[i, k]) < 1


def test_special_values():
    fr = M.frame(3, (0, 0, 0), (1, 1, 1), 0.25, 0.25)
    p = np.array([[0.0, 0.0, 0.0], [0.3, 0.7, 0.2], [0.3, 0.7, 0.2], [0.55, 0.7, 0.2]])
    X, c, q = M.fixed_point(p, (0, 0, 0), fr)
    assert float(q[0, 0]) == -1.0
    r2, _ = M.pair_r2_32(3, q[1:2], c[1:2], q[2:3], c[2:3])
    assert float(r2[0]) == 0.0
    # 0.25 apart along x = one cell width (times 1/(1 + 2^-30)): r2 = 4 (0.25 / w)^2
    r2, t = M.pair_r2_32(3, q[1:2], c[1:2], q[3:4], c[3:4])
    assert abs(float(r2[0]) - 4 * (0.25 / fr["w"]) ** 2) < 2 ** -20
    assert float(t[0, 0]) < 0 and float(t[0, 1]) == 0.0
    assert float(fr["t_lo"]) <= 4 * (fr["rho2"] - M.BAND) and float(fr["t_hi"]) >= 4 * (fr["rho2"] + M.BAND)
    assert float(fr["t_lo"]) < float(fr["t_mid"]) < float(fr["t_hi"])
    assert all(np.asarray(fr[k]).dtype == np.float32 for k in ("t_lo", "t_hi", "t_mid"))


@pytest.mark.parametrize("dim", [2, 3])
def test_r2_error_within_bound(dim):
    """Pairs across adjacent cells, concentrated near the cutoff: |r2_32 - 4 |delta|^2| is
    within the stated bound (exact rationals), and the bound within the band."""
    ps = W.ring_pairs(4000, 0.05, seed=dim, dim=dim, exps=(3, 5, 7, 9))
    fr = M.frame(dim, ps.lo, ps.hi, ps.cell_size, ps.radius)
    X, c, q = M.fixed_point(ps.pos, ps.lo, fr)
    i = np.arange(0, ps.n, 2)
    j = i + 1
    r2s, _ = M.pair_r2_32(dim, q[i], c[i], q[j], c[j])
    w = Fraction(fr["w"])
    worst = 0.0
    for a, b, v in zip(i, j, r2s):
        ex = 4 * sum((Fraction(float(ps.pos[b, k])) - Fraction(float(ps.pos[a, k]))) ** 2 for k in range(dim)) / w ** 2
        if ex <= 4 * Fraction(fr["rho2"]) * Fraction(5, 4):
            worst = max(worst, float(abs(Fraction(float(v)) - ex)))
    assert worst <= M.bound_r2(dim, fr["F"])
    assert worst > 0  # the test sees rounding at all
    assert M.bound_r2(dim, 20) < 4 * M.BAND


@pytest.mark.parametrize("maker", [
    lambda: W.lattice(2, 120, 1 / 120, 0.1, seed=1),
    lambda: W.lattice(3, 24, 1 / 24, 0.1, seed=2),
    lambda: W.uniform(2, 20000, seed=3),
    lambda: W.clustered(6000, 4, dim=3),
    lambda: W.ring_pairs(3000, 0.04, seed=5, dim=3),
    lambda: W.ring_pairs(3000, 0.03, seed=6, dim=2),
], ids=["lat2d", "lat3d", "uni2d", "clu3d", "ring3d", "ring2d"])
def test_three_way_test_reproduces_oracle(maker):
    """in / band-recheck / out gives exactly the oracle's neighbour count, nothing lands on
    the wrong side of the band, and FP32 is far more accurate than FP16 on the same pairs."""
    ps = maker()
    st = M.stats(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    s16 = M16.stats(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
    rp, _, _ = oracle.search_ps(ps)
    assert st["misplaced"] == 0
    assert st["nnz"] == rp[-1]
    assert st["candidates"] == s16["candidates"]
    assert st["band_pairs"] >= st["fp32_false_pos"] + st["fp32_false_neg"]
    assert st["band_pairs"] < s16["band_pairs"]
    assert st["fp32_false_pos"] + st["fp32_false_neg"] <= s16["fp16_false_pos"] + s16["fp16_false_neg"]
    assert st["max_err"] * 256 < max(s16["max_err"], 2.0 ** -30)
