"""Bit-level CPU model of the FP32 relative-coordinate test (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this
module. It shares no code with the GPU path. The paper studies its relative-coordinate
link list in FP32 as well as FP16 (Mixed-precision SPH, low-precision NNPS; the FP32
columns of the accuracy and timing comparisons): the cell and the coordinate inside the
cell are those of Eq. 6, the pair distance that of Eq. 7, only the floating-point format
of the stored coordinate and of the distance arithmetic changes.

The frame (cell width w, fraction bits F, fixed point X, cells c, D) is the one of the
FP16 model (same definitions, reused from it). FP32 specifics:
  q_k = f32(D_k) * 2^(1-F)                   (exact scaling of a rounded-to-nearest f32)
Per candidate j of target i, dc_k = c_i,k - c_j,k, every step rounded to f32, no fused
operations:
  t_k = (q_i,k - q_j,k) + 2 dc_k             (each axis alike)
  r2  = (t_x^2 + t_y^2) [+ t_z^2]            (squares rounded, sums left to right)
Thresholds on r2 (= 4 |delta|^2), rho2 = fl(fl(R/w)^2):
  T_lo = max(0, RD32(4 (rho2 - BAND))), T_hi = RU32(4 (rho2 + BAND)), T_mid = RN32(4 rho2)
  in <=> r2 < T_lo;  out <=> r2 > T_hi;  otherwise decided by the FP64 predicate.

Reading: the paper gives no op order for FP32; this one (each axis alike, no fusion) is
this library's, chosen so that numpy's correctly rounded float32 operations reproduce
it exactly.

BAND = 2^-15 squared cell widths. Bound (pinned in the tests against exact rational
arithmetic): the fixed point is within one unit 2^-F of the exact position (rint plus
the two binary64 roundings of fl(fl(p - lo) s) at magnitude < 2^51), i.e. 2^(1-F) in
q units; the f32 rounding of q adds at most 2^-25; with F >= 20 the two particles
contribute 2^-18 + 2^-24 to t, the subtraction (|.| < 2) 2^-24 and the addition of 2 dc
(|.| < 4) 2^-23: |t - 2 delta_k| <= e = 2^-18 + 2^-22 + 2^-24. Near the cutoff
|2 delta_k| <= 2, so |t^2 - 4 delta_k^2| <= e (4 + e) per axis, and the d squares and
d - 1 sums rounded at magnitude < 8 add at most (2d - 1) 2^-22: in all at most
12 e (1 + e/4) + 5 * 2^-22 < 2^-13 = 4 BAND on r2 in 3D.
"""
from __future__ import annotations

import numpy as np

from .rcll_fp16 import candidate_pairs, frame as frame16, r2_64

BAND = 2.0 ** -15


def rd32(x: float) -> np.float32:
    h = np.float32(x)
    if float(h) > x:
        h = np.nextafter(h, np.float32(-np.inf))
    return h


def ru32(x: float) -> np.float32:
    h = np.float32(x)
    if float(h) < x:
        h = np.nextafter(h, np.float32(np.inf))
    return h


def frame(dim, lo, hi, cell_size, radius):
    """The FP16 model's frame with the FP32 thresholds in place of the FP16 ones."""
    fr = dict(frame16(dim, lo, hi, cell_size, radius))
    rho2 = fr["rho2"]
    t_lo = rd32(4.0 * (rho2 - BAND))
    if float(t_lo) < 0.0:
        t_lo = np.float32(0.0)
    fr.update(t_lo=t_lo, t_hi=ru32(4.0 * (rho2 + BAND)), t_mid=np.float32(4.0 * rho2))
    return fr


def fixed_point(pos, lo, fr):
    """X (int64 [n, dim]), cells c, and the FP32 relative coordinates q (Eq. 6 scale)."""
    pos = np.asarray(pos, dtype=np.float64)
    n, dim = pos.shape
    F = fr["F"]
    d = pos - np.asarray(lo[:dim], dtype=np.float64)[None, :]
    X = np.rint(d * fr["s"]).astype(np.int64)
    c = X >> F
    D = X - (c << F) - (1 << (F - 1))
    q = D.astype(np.float32) * np.float32(2.0 ** (1 - F))
    return X, c, q


def pair_r2_32(dim, qi, ci, qj, cj):
    """FP32 r2 (4 |delta|^2) for arrays of pairs, each operation rounded to f32."""
    two_dc = (2 * (ci - cj)).astype(np.float32)  # small integers: exact
    t = (qi.astype(np.float32) - qj.astype(np.float32)) + two_dc
    sq = t * t
    r2 = sq[:, 0] + sq[:, 1]
    if dim == 3:
        r2 = r2 + sq[:, 2]
    return r2.astype(np.float32), t


def stats(pos, lo, hi, cell_size, radius, targets=None):
    """FP32-pass statistics over all candidates of the given targets (default: all), as
    the FP16 model's: candidates, band pairs, naive-FP32 false positives / negatives
    (r2 <= T_mid against the FP64 predicate), neighbour count, misplaced pairs (must be
    0), largest |r2_32/4 - r2_exact| (squared cell widths) within 2x the radius."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    fr = frame(dim, lo, hi, cell_size, radius)
    X, c, q = fixed_point(pos, lo, fr)
    R2 = radius * radius
    t_lo, t_hi, t_mid = float(fr["t_lo"]), float(fr["t_hi"]), float(fr["t_mid"])
    w = fr["w"]
    out = dict(candidates=0, band_pairs=0, fp32_false_pos=0, fp32_false_neg=0, nnz=0, misplaced=0,
               max_err=0.0)
    for ii, jj in candidate_pairs(c, fr["nc"], targets):
        r2s, _ = pair_r2_32(dim, q[ii], c[ii], q[jj], c[jj])
        r2s = r2s.astype(np.float64)
        truth = r2_64(pos[ii], pos[jj]) <= R2
        naive = r2s <= t_mid
        band = (r2s >= t_lo) & (r2s <= t_hi)
        inn = r2s < t_lo
        out["candidates"] += int(ii.size)
        out["band_pairs"] += int(band.sum())
        out["fp32_false_pos"] += int((naive & ~truth).sum())
        out["fp32_false_neg"] += int((~naive & truth).sum())
        out["nnz"] += int((inn | (band & truth)).sum())
        out["misplaced"] += int((inn & ~truth).sum() + (~inn & ~band & truth).sum())
        ex = r2_64(pos[ii], pos[jj]) / (w * w)
        near = ex <= 4.0 * (radius / w) ** 2
        if near.any():
            out["max_err"] = max(out["max_err"], float(np.max(np.abs(r2s[near] / 4.0 - ex[near]))))
    out.update(frame=fr)
    return out


def bound_r2(dim: int, F: int) -> float:
    """The bound of the module doc on |r2_32 - 4 |delta|^2| near the cutoff (r2 units),
    for fraction bits F."""
    e = 2.0 ** (1 - F) * 2 + 2.0 ** -22 + 2.0 ** -24
    return dim * 4.0 * e * (1.0 + e / 4.0) + (2 * dim - 1) * 2.0 ** -22


assert bound_r2(3, 20) < 4.0 * BAND  # the band covers the bound at the smallest F
