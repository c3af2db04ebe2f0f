"""Bit-level CPU model of the FP16 relative-coordinate test (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this
module. It shares no code with the GPU path; it restates, in numpy, the documented
arithmetic of the FP16 pass so that its statistics (candidates, band pairs, FP16
false positives and negatives before the FP64 recheck) can be compared bit for bit.

Paper sources:
  * Eq. 5 normalises the domain and Eq. 6 stores each particle's coordinate relative
    to its cell centre, scaled into [-1, 1] (Mixed-precision SPH, low-precision NNPS).
  * Eq. 7 recovers a pair's distance from the two relative coordinates plus the
    offset between the two cell centres.

Readings (where the paper is silent or garbled):
  * Eq. 7 as printed drops a factor 1/2: with Eq. 6 the displacement in cell-width
    units is (q_i - q_j)/2 + (c_i - c_j). The model works with twice that, so that
    t = (q_i - q_j) + 2(c_i - c_j) and the squared norm is 4 |delta|^2.
  * Eq. 5 cancels when Eq. 6 is applied on top of it (only the cell width matters),
    so the cell and the relative coordinate come from one fixed-point value
    X = rint((p - lo) * 2^F / w) instead of from normalised FP64 coordinates.
  * The cell centres are kept as integer cell indices, so the centre offset is exact.
  * FP16 rounding error alone cannot give an exact neighbour set, so each FP16 r^2
    within a guard band of the cutoff is decided again in FP64 (this library's
    addition; the band is BAND = 2^-7 in units of the squared cell width).

The fixed definitions (identical on the GPU):
  w   = fl(max(cell_size, R) * (1 + 2^-30))
  F   = min(40, 51 - bitlen(max_k floor((hi_k - lo_k)/w) + 1))
  X_k = rint(fl(fl(p_k - lo_k) * fl(2^F / w)))        (round half to even, int64)
  nc_k = (X_k(hi_k) >> F) + 1;  c_k = X_k >> F
  D_k = X_k - c_k 2^F - 2^(F-1);  q_k = f16(f32(D_k) * 2^(1-F))      (Eq. 6 scale)
Per candidate j of target i (dc_k = c_i,k - c_j,k), every step rounded to f16:
  x:    s = q_i,x - q_j,x;   t_x = s + 2 dc_x
  y, z: A_k = q_i,k + 2 dc_k;  t_k = A_k - q_j,k
  r2 = t_z^2; r2 = fma(t_y, t_y, r2); r2 = fma(t_x, t_x, r2)     (2D: no z term)
Thresholds on r2 (= 4 |delta|^2), rho2 = fl(fl(R/w)^2):
  T_lo = max(0, RD16(4 (rho2 - BAND))), T_hi = RU16(4 (rho2 + BAND)), T_mid = RN16(4 rho2)
  in  <=> r2 < T_lo;  out <=> r2 > T_hi;  otherwise FP64 recheck.
The naive FP16 decision (r2 <= T_mid) is what the misclassification counts measure.
"""
from __future__ import annotations

import math

import numpy as np

BAND = 2.0 ** -7


def rd16(x: float) -> np.float16:
    """Largest f16 <= x."""
    h = np.float16(x)
    if float(h) > x:
        h = np.nextafter(h, np.float16(-np.inf))
    return h


def ru16(x: float) -> np.float16:
    """Smallest f16 >= x."""
    h = np.float16(x)
    if float(h) < x:
        h = np.nextafter(h, np.float16(np.inf))
    return h


def frame(dim, lo, hi, cell_size, radius):
    """Cell width, fraction bits, scale, cell counts and thresholds (see module doc)."""
    w = max(cell_size, radius) * (1.0 + 2.0 ** -30)
    ncest = [math.floor((hi[k] - lo[k]) / w) + 1 for k in range(dim)]
    F = min(40, 51 - int(max(ncest)).bit_length())
    s = math.ldexp(1.0, F) / w
    nc = []
    for k in range(dim):
        xh = int(np.rint((hi[k] - lo[k]) * s))
        nc.append((xh >> F) + 1)
    rho = radius / w
    rho2 = rho * rho
    t_lo = rd16(4.0 * (rho2 - BAND))
    if float(t_lo) < 0.0:
        t_lo = np.float16(0.0)
    t_hi = ru16(4.0 * (rho2 + BAND))
    t_mid = np.float16(4.0 * rho2)
    return dict(w=w, F=F, s=s, nc=nc, rho2=rho2, t_lo=t_lo, t_hi=t_hi, t_mid=t_mid)


def fixed_point(pos, lo, fr):
    """X (int64 [n, dim]), cells c, and the FP16 relative coordinates q (Eq. 6 scale)."""
    pos = np.asarray(pos, dtype=np.float64)
    n, dim = pos.shape
    F = fr["F"]
    d = pos - np.asarray(lo[:dim], dtype=np.float64)[None, :]
    X = np.rint(d * fr["s"]).astype(np.int64)
    c = X >> F
    D = X - (c << F) - (1 << (F - 1))
    q = (D.astype(np.float32) * np.float32(2.0 ** (1 - F))).astype(np.float16)
    return X, c, q


def _f16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16)


def pair_r2_16(dim, qi, ci, qj, cj):
    """FP16 r2 (4 |delta|^2) for arrays of pairs; each step rounded to f16 as documented."""
    dc = (ci - cj).astype(np.float64)
    s = _f16(qi[:, 0].astype(np.float64) - qj[:, 0].astype(np.float64))
    tx = _f16(s.astype(np.float64) + 2.0 * dc[:, 0])
    ay = _f16(qi[:, 1].astype(np.float64) + 2.0 * dc[:, 1])
    ty = _f16(ay.astype(np.float64) - qj[:, 1].astype(np.float64))
    if dim == 3:
        az = _f16(qi[:, 2].astype(np.float64) + 2.0 * dc[:, 2])
        tz = _f16(az.astype(np.float64) - qj[:, 2].astype(np.float64))
        tz64 = tz.astype(np.float64)
        r2 = _f16(tz64 * tz64)
        ty64 = ty.astype(np.float64)
        r2 = _f16(ty64 * ty64 + r2.astype(np.float64))
    else:
        ty64 = ty.astype(np.float64)
        r2 = _f16(ty64 * ty64)
    tx64 = tx.astype(np.float64)
    r2 = _f16(tx64 * tx64 + r2.astype(np.float64))
    return r2, np.stack([tx, ty] + ([tz] if dim == 3 else []), axis=1)


def r2_64(pos_i, pos_j):
    """The oracle's FP64 r2 in its fixed order, vectorised (numpy does not fuse)."""
    d0 = pos_j[:, 0] - pos_i[:, 0]
    d1 = pos_j[:, 1] - pos_i[:, 1]
    r2 = d0 * d0
    r2 = r2 + d1 * d1
    if pos_i.shape[1] == 3:
        d2 = pos_j[:, 2] - pos_i[:, 2]
        r2 = r2 + d2 * d2
    return r2


def candidate_pairs(c, nc, targets=None):
    """All (i, j), j != i, with j in the clipped 3^d block of cells around i's cell.
    Yields chunks of (i, j) index arrays."""
    n, dim = c.shape
    key = c[:, 0] + nc[0] * c[:, 1]
    if dim == 3:
        key = key + nc[0] * nc[1] * c[:, 2]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    ncell = int(np.prod(nc))
    cs = np.searchsorted(skey, np.arange(ncell + 1), side="left")
    if targets is None:
        targets = np.arange(n)
    offs = [(a, b, e) for e in ((-1, 0, 1) if dim == 3 else (0,)) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    chunk = 1 << 16
    for t0 in range(0, len(targets), chunk):
        ti = targets[t0:t0 + chunk]
        ct = c[ti]
        for (a, b, e) in offs:
            cx = ct[:, 0] + a
            cy = ct[:, 1] + b
            ok = (cx >= 0) & (cx < nc[0]) & (cy >= 0) & (cy < nc[1])
            k = cx + nc[0] * cy
            if dim == 3:
                cz = ct[:, 2] + e
                ok &= (cz >= 0) & (cz < nc[2])
                k = k + nc[0] * nc[1] * cz
            k = np.where(ok, k, 0)
            start = np.where(ok, cs[k], 0)
            cnt = np.where(ok, cs[np.minimum(k + 1, ncell)] - cs[k], 0)
            tot = int(cnt.sum())
            if tot == 0:
                continue
            ii = np.repeat(ti, cnt)
            base = np.repeat(start - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
            jj = order[base + np.arange(tot)]
            keep = jj != ii
            yield ii[keep], jj[keep]


def stats(pos, lo, hi, cell_size, radius, targets=None):
    """FP16-pass statistics over all candidates of the given targets (default: all):
    candidates, band pairs, naive-FP16 false positives / negatives, neighbour count,
    pairs the three-way test misplaces (must be 0), the largest |r2_16/4 - r2_exact| in
    squared cell widths among pairs within 2x the radius, and the largest ratio of that
    error to `error_bound` at the pair's distance (must be <= 1)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    fr = frame(dim, lo, hi, cell_size, radius)
    X, c, q = fixed_point(pos, lo, fr)
    R2 = radius * radius
    t_lo = float(fr["t_lo"])
    t_hi = float(fr["t_hi"])
    t_mid = float(fr["t_mid"])
    w = fr["w"]
    out = dict(candidates=0, band_pairs=0, fp16_false_pos=0, fp16_false_neg=0, nnz=0,
               misplaced=0, max_err=0.0, max_err_ratio=0.0)
    for ii, jj in candidate_pairs(c, fr["nc"], targets):
        r2h, _ = pair_r2_16(dim, q[ii], c[ii], q[jj], c[jj])
        r2h = r2h.astype(np.float64)
        truth = r2_64(pos[ii], pos[jj]) <= R2
        naive = r2h <= t_mid
        band = (r2h >= t_lo) & (r2h <= t_hi)
        inn = r2h < t_lo
        out["candidates"] += int(ii.size)
        out["band_pairs"] += int(band.sum())
        out["fp16_false_pos"] += int((naive & ~truth).sum())
        out["fp16_false_neg"] += int((~naive & truth).sum())
        out["nnz"] += int((inn | (band & truth)).sum())
        out["misplaced"] += int((inn & ~truth).sum() + (~inn & ~band & truth).sum())
        ex = r2_64(pos[ii], pos[jj]) / (w * w)
        near = ex <= 4.0 * (radius / w) ** 2
        if near.any():
            err = np.abs(r2h[near] / 4.0 - ex[near])
            out["max_err"] = max(out["max_err"], float(np.max(err)))
            ratio = err / error_bound(dim, np.sqrt(ex[near]))
            out["max_err_ratio"] = max(out["max_err_ratio"], float(np.max(ratio)))
    out.update(frame=fr)
    return out


def error_bound(dim, delta):
    """A bound on |r2_16/4 - |delta|^2| (squared cell widths) for a pair at true distance
    delta (cell widths), for the documented op sequence.

    Per component, in units of 2 delta: storage of each q is within 2^-12 (f32 then f16
    rounding), each of the two f16 steps adds at most half an ulp at magnitude < 4
    (2^-10); so |t - 2 delta_k| <= 2^-11 + 2 * 2^-10 + 2^-20 = e2. Then
    |t^2 - 4 delta_k^2| <= e2 (4 |delta_k| + e2), and the chain of d roundings adds at
    most d half-ulps relative (2^-11 each) of partial sums bounded by the final sum."""
    e2 = 2.0 ** -11 + 2 * 2.0 ** -10 + 2.0 ** -20
    lin = e2 * (4.0 * math.sqrt(dim) * np.asarray(delta) + dim * e2)
    total = 4.0 * delta * delta + lin
    chain = dim * 2.0 ** -11 * total * 1.0001
    b = (lin + chain) / 4.0
    return float(b) if np.ndim(b) == 0 else b
