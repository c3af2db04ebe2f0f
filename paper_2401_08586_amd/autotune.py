"""Autotuner for the library's work shapes (nnps_tuning): block size target of the block
path, the stencil size above which windows take the dense-cell path, and the workgroup
counts of the dense and long-row kernels.

The tuner times whole build + count + fill steps (HIP events around the library's batch
step) on the caller's own sets, one knob at a time (coordinate descent from the defaults,
two sweeps), and keeps the fastest setting. Results are cached in a JSON file keyed by the
device architecture, dimension, mode and a coarse description of the workload (total
particles and the spread of stencil sizes, both as powers of two), so a later call on a
similar workload reuses them without timing.

The search (`coordinate_descent`) and the cache are host logic, tested on the CPU with a
stand-in cost function.
"""
from __future__ import annotations

import json
import math
import os

DEFAULTS = {"block_target": 80, "long_rows_grid": 1024, "long_rows_keys": 0, "dense_min_union": 0,
            "dense_grid": 0, "dense_max_entries": 0}

SPACE = {
    "block_target": [32, 48, 56, 64, 72, 80, 88, 96],
    "dense_min_union": [1, 128, 256, 384, 512, 768, 1024, -1],
    "dense_grid": [256, 512, 1024, 1280, 2048, 4096],
    "long_rows_grid": [256, 1024, 4096],
}


def coordinate_descent(cost, space=None, start=None, sweeps: int = 2):
    """Minimise cost(params) one knob at a time over `space` ({knob: [values]}), starting
    from `start`; each sweep visits every knob in order and keeps the best value found.
    Returns (best params, best cost, number of evaluations). Costs are cached per setting."""
    space = space or SPACE
    cur = dict(start or DEFAULTS)
    seen = {}

    def f(p):
        key = tuple(sorted(p.items()))
        if key not in seen:
            seen[key] = cost(dict(p))
        return seen[key]

    best = f(cur)
    for _ in range(sweeps):
        changed = False
        for knob, values in space.items():
            for v in values:
                if cur.get(knob) == v:
                    continue
                trial = dict(cur)
                trial[knob] = v
                c = f(trial)
                if c < best:
                    best, cur, changed = c, trial, True
        if not changed:
            break
    return cur, best, len(seen)


def workload_key(arch: str, dim: int, mode: int, sizes, stencil_p99: float, stencil_mean: float) -> str:
    """A coarse key: total particles and set count as powers of two, stencil-size spread
    (p99 / mean) as a power of two and the mean stencil size as a power of two."""
    n = max(1, int(sum(sizes)))
    return (f"{arch}|d{dim}|m{mode}|n2^{int(math.log2(n))}|s2^{int(math.log2(max(1, len(sizes))))}"
            f"|u2^{int(math.log2(max(1.0, stencil_mean)))}"
            f"|spread2^{int(math.log2(max(1.0, stencil_p99 / max(stencil_mean, 1e-9))))}")


class Cache:
    """{key: {"params": {...}, "ms": best}} in a JSON file (written atomically)."""

    def __init__(self, path: str | None = None):
        self.path = path or os.path.join(os.path.expanduser("~"), ".cache", "nnps_autotune.json")
        self.data = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key):
        e = self.data.get(key)
        return dict(e["params"]) if e else None

    def put(self, key, params, ms):
        self.data[key] = {"params": dict(params), "ms": float(ms)}
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def stencil_sizes(ps_list, sample: int = 20000, seed: int = 0):
    """Mean and p99 of the number of particles in a particle's 3^d cell stencil, estimated
    on the host from a sample of each set (only to key the cache)."""
    import itertools

    import numpy as np
    rng = np.random.default_rng(seed)
    vals = []
    for ps in ps_list:
        if ps.n == 0:
            continue
        d = ps.dim
        w = max(ps.cell_size, ps.radius)
        c = np.floor((ps.pos - np.asarray(ps.lo, dtype=np.float64)) / w).astype(np.int64)
        nc = c.max(axis=0) + 1
        mul = np.array([1, nc[0], nc[0] * nc[1]][:d], dtype=np.int64)
        occ = np.bincount(c @ mul, minlength=int(np.prod(nc)))
        ci = c[rng.choice(ps.n, size=min(sample, ps.n), replace=False)]
        tot = np.zeros(len(ci), dtype=np.int64)
        for off in itertools.product((-1, 0, 1), repeat=d):
            q = ci + np.asarray(off)
            ok = np.all((q >= 0) & (q < nc), axis=1)
            tot[ok] += occ[q[ok] @ mul]
        vals.append(tot)
    if not vals:
        return 0.0, 0.0
    v = np.concatenate(vals).astype(np.float64)
    return float(v.mean()), float(np.percentile(v, 99))


def tune(ctx, sets, pss=None, mode: int = 0, steps: int = 3, warmup: int = 1, space=None, cache: Cache | None = None,
         use_cache: bool = True, log=None, sweeps: int = 2):
    """Pick nnps_tuning for `sets` (list of (pos, lo, hi, cell_size, radius) device sets);
    `pss` (workloads.ParticleSet list of the same sets) keys the cache. Leaves the chosen
    tuning set on `ctx` and returns (params, ms per step, evaluations)."""
    import torch
    from . import nnps
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    key = None
    if pss is not None and use_cache:
        mean, p99 = stencil_sizes(pss, sample=2000)
        key = workload_key(arch, sets[0][0].shape[1], mode, [p.n for p in pss], p99, mean)
        cache = cache or Cache()
        hit = cache.get(key)
        if hit is not None:
            ctx.set_tuning(**hit)
            return hit, None, 0
    rps = [torch.empty(s[0].shape[0] + 1, dtype=torch.int64, device="cuda") for s in sets]
    probe = ctx.cells()
    probe.batch_build(sets, mode)
    nnz = probe.batch_count(rps, sync=True)
    probe.close()
    cols = [torch.empty(max(k, 1), dtype=torch.int32, device="cuda") for k in nnz]
    dists = [torch.empty(max(k, 1), dtype=torch.float32, device="cuda") for k in nnz]
    stream = torch.cuda.Stream()
    cells = ctx.cells()  # one structure for every trial: its buffers are reused

    def cost(p):
        ctx.set_tuning(**p)
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                cells.batch_step(sets, rps, cols, dists, mode, stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                cells.batch_step(sets, rps, cols, dists, mode, stream=stream)
            e1.record(stream)
        got = cells.batch_nnz(stream=stream)
        if got != nnz:
            raise RuntimeError(f"tuning {p} changed the neighbour counts")
        ms = e0.elapsed_time(e1) / steps
        if log:
            log(f"[autotune] {p} -> {ms:.3f} ms")
        return ms

    try:
        best, ms, evals = coordinate_descent(cost, space=space, sweeps=sweeps)
    finally:
        cells.close()
    ctx.set_tuning(**best)
    if key is not None:
        cache.put(key, best, ms)
    return best, ms, evals
