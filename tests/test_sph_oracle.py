"""Pins of the SPH-gradient oracle (oracle/sph_gradient.py) against what the paper and the
mathematics fix: the kernel's normalisation and derivative (Eq. 3), the exactness of the
normalised operator (Eq. A5) on linear fields, closed-form lattice sums for f = x^3 and
for Eq. 2 on f = x, and the first-order error trend of Table 3."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import sph_gradient as G
from paper_2401_08586_amd import workloads as W


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_integrates_to_one(dim):
    """alpha_d of Eq. 3 normalises W over its support (ring / shell measure)."""
    h = 0.37
    meas = (lambda r: 2 * math.pi * r) if dim == 2 else (lambda r: 4 * math.pi * r * r)
    val, _ = integrate.quad(lambda r: float(G.kernel_w(r / h, dim, h)) * meas(r), 0.0, 2 * h, points=[h])
    assert abs(val - 1.0) < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_derivative_matches_finite_differences(dim):
    h = 0.5
    r = np.linspace(0.01, 1.2, 97)
    r = r[np.abs(r - h) > 1e-3]  # away from the knot at R = 1 (continuous derivative, kink in W'')
    eps = 1e-6
    fd = (G.kernel_w((r + eps) / h, dim, h) - G.kernel_w((r - eps) / h, dim, h)) / (2 * eps)
    assert np.allclose(G.kernel_dwdr(r, dim, h), fd, rtol=1e-6, atol=1e-7)
    assert np.all(G.kernel_dwdr(np.array([2 * h, 3 * h]), dim, h) == 0.0)


def _csr(ps, radius=None):
    return oracle.search(ps.pos, ps.lo, ps.hi, ps.cell_size, radius or ps.radius)


@pytest.mark.parametrize("dim", [2, 3])
def test_normalised_operator_is_exact_on_linear_fields(dim):
    """Eq. A5 works axis by axis: for f = c + a x_k, axis k of every row with a non-zero
    denominator returns a (up to rounding), whatever the neighbour set (numerator = a times
    the denominator term by term). Rows without neighbours return 0."""
    ps = W.uniform(dim, 3000 if dim == 2 else 4000, seed=5)
    rp, col, _ = _csr(ps)
    h = ps.radius / 2.0
    has = np.diff(rp) > 0
    assert has.sum() > 0.9 * ps.n
    for k, a in enumerate((2.0, -5.0, 0.5)[:dim]):
        f = 3.0 + a * ps.pos[:, k]
        _, norm, _ = G.gradient(ps.pos, f, h, rp, col)
        assert np.allclose(norm[has, k], a, rtol=1e-9, atol=1e-9)
        assert np.all(norm[~has] == 0.0)


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 14)])
def test_lattice_closed_forms(dim, n):
    """Perfect lattice, interior sites: Eq. A5 on f = x^3 gives 3x^2 + dx^2 S4/S2 and 0 on the
    other axes; Eq. 2 on f = x with V = dx^d gives -dx^(d+2) sum g o_x^2, within 2 % of the
    continuum value 1 (a check of alpha_d)."""
    dx = 1.0 / n
    ps = W.lattice(dim, n, dx, jitter=0.0)
    rp, col, _ = _csr(ps)
    h = 1.2 * dx
    x = ps.pos[:, 0]
    _, norm, _ = G.gradient(ps.pos, x ** 3, h, rp, col)
    std, _, _ = G.gradient(ps.pos, x.copy(), h, rp, col, vol=np.full(ps.n, dx ** dim))
    margin = ps.radius + 1e-12
    interior = np.all((ps.pos > margin) & (ps.pos < 1.0 - margin), axis=1)
    assert interior.sum() > 0
    corr = G.lattice_ratio_x3(dim, dx, h, ps.radius)
    assert np.allclose(norm[interior, 0], 3 * x[interior] ** 2 + corr, rtol=1e-9, atol=1e-12)
    assert np.allclose(norm[interior, 1:], 0.0, atol=1e-9)
    lin = G.lattice_linear_std(dim, dx, h, ps.radius)
    assert abs(lin - 1.0) < 0.02
    assert np.allclose(std[interior, 0], lin, rtol=1e-9)
    assert np.allclose(std[interior, 1:], 0.0, atol=1e-9)


def test_cell_list_and_brute_force_lists_give_the_same_gradient():
    ps = W.clustered(1500, seed=2, dim=3)
    rp, col, _ = _csr(ps)
    rpb, colb, _ = oracle.search(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, brute=True)
    f = np.sin(7 * ps.pos[:, 0]) + ps.pos[:, 1] ** 2
    h = ps.radius / 2
    for a, b in zip(G.gradient(ps.pos, f, h, rp, col)[:2], G.gradient(ps.pos, f, h, rpb, colb)[:2]):
        assert np.array_equal(a, b)


def test_first_order_trend_of_table3():
    """Table 3: the RMSE of the Eq. A5 gradient of f = x^3 halves with the particle spacing.
    Uniform random points in the unit square, Delta s = (1/N)^(1/2), h = 1.2 Delta s."""
    rmse = []
    for npart in (2500, 10000):
        ps = W.uniform(2, npart, seed=11)
        rp, col, _ = _csr(ps)
        x = ps.pos[:, 0]
        _, norm, _ = G.gradient(ps.pos, x ** 3, ps.radius / 2, rp, col)
        rmse.append(float(np.sqrt(np.mean((norm[:, 0] - 3 * x ** 2) ** 2))))
    assert 1.5 < rmse[0] / rmse[1] < 2.7, rmse
