"""CPU oracle of the SPH gradient over a neighbour list (test infrastructure only).

Plain numpy in binary64, term by term as the paper defines it:

* the cubic B-spline kernel W(R, h) of Eq. 3 (SPH method section), R = r / h, support 2h,
  alpha_d = 15 / (7 pi h^2) in 2D and 3 / (2 pi h^3) in 3D; its gradient with respect to
  particle i is dW/dr * (x_i - x_j) / r, with dW/dr = alpha_d / h * dW/dR;
* the standard gradient approximation of Eq. 2: sum over the neighbours j of V_j f_j dW_ij;
* the normalised, volume-free first-order operator of the appendix (Eq. A5): per axis,
  sum_j (f_j - f_i) dW_ij / sum_j (x_j - x_i) dW_ij.

Besides the values, `gradient` returns per row and axis the sum of the absolute values of
the summed terms, from which a test bounds the rounding of any summation order.
"""
from __future__ import annotations

import math

import numpy as np


def alpha_d(dim: int, h: float) -> float:
    """Normalisation of the cubic B-spline (Eq. 3)."""
    if dim == 2:
        return 15.0 / (7.0 * math.pi * h * h)
    if dim == 3:
        return 3.0 / (2.0 * math.pi * h ** 3)
    raise ValueError("dim must be 2 or 3")


def kernel_w(R, dim: int, h: float):
    """W(R, h) of Eq. 3 (vectorised over R = r / h)."""
    R = np.asarray(R, dtype=np.float64)
    w = np.where(R < 1.0, 2.0 / 3.0 - R ** 2 + 0.5 * R ** 3,
                 np.where(R < 2.0, (2.0 - R) ** 3 / 6.0, 0.0))
    return alpha_d(dim, h) * w


def kernel_dwdr(r, dim: int, h: float):
    """dW/dr: Eq. 3 differentiated, dW/dR = -2R + 3/2 R^2 (R < 1), -(2 - R)^2 / 2 (1 <= R < 2),
    0 beyond, times alpha_d / h."""
    R = np.asarray(r, dtype=np.float64) / h
    dwdR = np.where(R < 1.0, -2.0 * R + 1.5 * R * R, np.where(R < 2.0, -0.5 * (2.0 - R) ** 2, 0.0))
    return alpha_d(dim, h) / h * dwdR


def gradient(pos, f, h, row_ptr, col, vol=None, targets=None):
    """Returns grad [m, d] (Eq. 2), grad_norm [m, d] (Eq. A5, 0 where the denominator is 0)
    and (abs_s, abs_num, abs_den, num, den), each [m, d]: the sums of the absolute values of
    the summed terms and the numerator and denominator of Eq. A5, for the m rows of the CSR
    (row_ptr [m+1], col): row k belongs to particle targets[k] (default: k)."""
    pos = np.asarray(pos, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    n, dim = pos.shape
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    vol = np.ones(n) if vol is None else np.asarray(vol, dtype=np.float64)
    m = len(row_ptr) - 1
    targets = np.arange(m) if targets is None else np.asarray(targets, dtype=np.int64)
    slot = np.repeat(np.arange(m), np.diff(row_ptr))   # CSR row of each entry
    rows = targets[slot]                                # its target particle
    dx = pos[col] - pos[rows]                                # x_j - x_i
    r = np.sqrt(np.sum(dx * dx, axis=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.where(r > 0.0, kernel_dwdr(r, dim, h) / r, 0.0)  # dW/dr / r
    dw = g[:, None] * (-dx)                                   # dW_ij / dx_i = dW/dr (x_i - x_j) / r
    t_s = (vol[col] * f[col])[:, None] * dw
    t_num = (f[col] - f[rows])[:, None] * dw
    t_den = dx * dw
    out = []
    for t in (t_s, t_num, t_den, np.abs(t_s), np.abs(t_num), np.abs(t_den)):
        acc = np.zeros((m, dim))
        np.add.at(acc, slot, t)
        out.append(acc)
    s, num, den, abs_s, abs_num, abs_den = out
    with np.errstate(divide="ignore", invalid="ignore"):
        norm = np.where(den != 0.0, num / den, 0.0)
    return s, norm, (abs_s, abs_num, abs_den, num, den)


def sum_bound(abs_sum, nterms):
    """Bound on the rounding error of summing terms whose absolute values sum to abs_sum,
    in any order, with each term itself within a few ulps: (nterms + 8) u sum |t|."""
    u = 2.0 ** -53
    return (np.asarray(nterms, dtype=np.float64)[:, None] + 8.0) * u * abs_sum


def lattice_ratio_x3(dim: int, dx: float, h: float, radius: float):
    """Closed form of the Eq. A5 x-derivative of f = x^3 at an interior site of a perfect
    lattice with spacing dx and neighbours within `radius`: every offset o comes with -o, so
    the odd moments cancel and the result is 3x^2 + dx^2 S4 / S2 with
    S_p = sum_o o_x^p g(|o| dx), g = dW/dr / r. Returns dx^2 S4 / S2."""
    m = int(math.floor(radius / dx)) + 1
    rng = range(-m, m + 1)
    s2 = s4 = 0.0
    for o in np.array(np.meshgrid(*([list(rng)] * dim), indexing="ij")).reshape(dim, -1).T:
        rr = float(np.sqrt(np.sum((o * dx) ** 2)))
        if rr == 0.0 or rr > radius:
            continue
        g = float(kernel_dwdr(rr, dim, h)) / rr
        s2 += g * o[0] ** 2
        s4 += g * o[0] ** 4
    return dx * dx * s4 / s2


def lattice_linear_std(dim: int, dx: float, h: float, radius: float):
    """Closed form of Eq. 2 for f = x with V = dx^d at an interior site of a perfect lattice:
    -dx^(d+2) sum_o g(|o| dx) o_x^2 (the continuum value is 1)."""
    m = int(math.floor(radius / dx)) + 1
    rng = range(-m, m + 1)
    s = 0.0
    for o in np.array(np.meshgrid(*([list(rng)] * dim), indexing="ij")).reshape(dim, -1).T:
        rr = float(np.sqrt(np.sum((o * dx) ** 2)))
        if rr == 0.0 or rr > radius:
            continue
        s += float(kernel_dwdr(rr, dim, h)) / rr * o[0] ** 2
    return -dx ** (dim + 2) * s
