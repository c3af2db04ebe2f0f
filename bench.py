#!/usr/bin/env python3
"""Neighbour-search throughput on one MI355X: FP16 relative-coordinate link list (with the
FP64 guard-band recheck) beside the plain FP64 GPU cell list and the CPU oracle.

One step = one whole search over the workload with the positions already in HBM:
cell build (FP64 assignment, radix sort, cell starts, FP16 pack, block table) + count
pass + row_ptr scan + fill pass. Output buffers are sized once from the warm-up count
(the workload is fixed), so the timed steps do not stop for the nnz read-back.
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one fill launch at the default workload, measured by rocprofv3 on the
# kernel source with this hash (profiles/k_fill_k_count_lattice3d_1M.md):
#   DRAM bytes: TCC_EA0_RDREQ_DRAM_32B_sum and TCC_EA0_WRREQ_WRITE_DRAM_32B_sum count
#     32-byte units of DRAM traffic; a 512 MiB device copy reads and writes exactly 2^24
#     of each (calibration factor 1.000);
#   FETCH_SIZE / WRITE_SIZE (KiB): the copy reads 262,144 KiB fetched and 524,288 KiB
#     written for 524,288 KiB moved each way, so they scale by 2.000 and 1.000.
# Reported only while the source is unchanged (the counters belong to that code).
FILL_TRAFFIC = {"source_sha256_16": "9cf6101d64cef744", "dram_read_bytes": 220.2e6, "dram_write_bytes": 487.3e6,
                "fetch_kib": 108373, "write_kib": 475898, "fetch_scale": 2.0, "write_scale": 1.0}


# VALU wave-instructions per launch (SQ_INSTS_VALU) of the C2 search kernels, from the
# profile of the same source; like the traffic, reported only while the source is unchanged
VALU_INSTS = {"source_sha256_16": "9cf6101d64cef744", "k_fill<3,0>": 136435229, "k_count16<3,0,false>": 129009217}


def valu_ceilings():
    """Measured VALU issue ceilings (wave64 instructions/s) of this device: long runs of
    independent packed-FP16 fma, FP32 fma and 32-bit integer instructions
    (nnps_probe_valu_rate)."""
    from paper_2401_08586_amd import nnps
    out = {}
    for kind in nnps.PROBE_KINDS:
        rate, per_wave = nnps.probe_valu_rate(kind)
        out[kind] = rate
    return out


def issue_rates(ph, ceilings):
    """Achieved VALU issue rate of the fill and count kernels (wave-instructions/s) from the
    profiled instruction counts and this run's mean launch times, against the measured
    32-bit integer ceiling, or None if the source changed since the profile."""
    import hashlib
    src = os.path.join(ROOT, "paper_2401_08586_amd", "csrc", "search_kernels.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != VALU_INSTS["source_sha256_16"]:
            return None
    out = {}
    # the kernels' instructions are 32-bit integer and bit work plus packed FP16 (the count's
    # FP16 share is about a quarter); FP32's dual issue does not apply to them
    peak = ceilings["int32"]
    for k, phase in (("k_fill<3,0>", "fill"), ("k_count16<3,0,false>", "count")):
        rate = VALU_INSTS[k] / (ph[phase] * 1e-3)
        out[k] = {"valu_insts_per_launch": VALU_INSTS[k], "avg_launch_ms": ph[phase], "achieved": rate,
                  "peak": peak, "peak_kind": "measured 32-bit integer issue rate (nnps_probe_valu_rate)",
                  "unit": "VALU wave-instructions/s", "frac": rate / peak}
    return out


def measured_copy_gbs(nbytes=1 << 29, reps=10):
    """HBM bandwidth a plain device-to-device copy reaches (bytes read + written per second,
    HIP events around `reps` copies of `nbytes`): the practical ceiling beside the datasheet
    peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def fill_traffic():
    """Measured fill traffic per launch if the search kernels are unchanged since the profile:
    DRAM bytes (read + write) and the FETCH_SIZE/WRITE_SIZE reading scaled by the copy."""
    import hashlib
    src = os.path.join(ROOT, "paper_2401_08586_amd", "csrc", "search_kernels.hip")
    with open(src, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    if h != FILL_TRAFFIC["source_sha256_16"]:
        return None, None
    t = FILL_TRAFFIC
    dram = t["dram_read_bytes"] + t["dram_write_bytes"]
    fw = (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024
    return dram, {"dram_read_bytes": t["dram_read_bytes"], "dram_write_bytes": t["dram_write_bytes"],
                  "fetch_write_size_bytes": fw, "source_sha256_16": h}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2401_08586_amd import workloads as W
    return {"c0": W.c0, "c1": W.c1, "c2": W.c2}[name]()


def describe(ps):
    return {"workload": ps.name, "particles": ps.n, "dim": ps.dim, "radius": ps.radius,
            "cell_size": ps.cell_size, "box": [list(ps.lo), list(ps.hi)],
            "inputs": "jittered lattice, dx = radius/2.4, jitter U(+-0.1 dx), seeded"}


def time_mode(ctx, pos, ps, mode, steps, warmup):
    """Returns (ms per step, nnz, stats, per-phase mean ms) for one mode: the timed steps
    replay the captured build + count + fill of the set (no events inside), and the
    per-phase means come from as many eager steps with an event pair around each phase."""
    ms, nnz, st, phases = time_batch(ctx, [ps], mode, steps, warmup, pos=[pos], phase_steps=steps)
    return ms, nnz, st, phases


def time_batch(ctx, pss, mode, steps, warmup, graphs=True, pos=None, phase_steps=1, half=False):
    """Batch of particle sets: one graph-captured step (build + count + fill) per timed
    step. Returns (ms per step, total nnz, stats, per-phase mean ms over `phase_steps`
    further eager steps)."""
    import torch
    from paper_2401_08586_amd import nnps
    if pos is None:
        pos = [torch.from_numpy(p.pos).cuda() for p in pss]
    sets = [(x, p.lo, p.hi, p.cell_size, p.radius) for x, p in zip(pos, pss)]
    cells = ctx.cells()
    cells.set_half(half)
    cells.batch_build(sets, mode)
    rps = [torch.empty(p.n + 1, dtype=torch.int64, device="cuda") for p in pss]
    nnz = cells.batch_count(rps, sync=True)
    cols = [torch.empty(k, dtype=torch.int32, device="cuda") for k in nnz]
    dists = [torch.empty(k, dtype=torch.float32, device="cuda") for k in nnz]
    cells.batch_fill(rps, cols, dists)
    st = cells.stats()
    stream = torch.cuda.Stream()
    cells.set_graphs(graphs)
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            cells.batch_step(sets, rps, cols, dists, mode, stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            cells.batch_step(sets, rps, cols, dists, mode, stream=stream)
        e1.record(stream)
        stream.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    assert cells.batch_nnz(stream=stream) == nnz
    # per-phase times of further eager steps
    cells.set_graphs(False)
    cells.set_profiling(True)
    with torch.cuda.stream(stream):
        for _ in range(max(1, phase_steps)):
            cells.batch_step(sets, rps, cols, dists, mode, stream=stream)
    ph = cells.phase_times(stream=stream)
    cells.set_profiling(False)
    cells.close()
    del cols, dists
    torch.cuda.empty_cache()
    return (max(wall, e0.elapsed_time(e1)) / steps, int(sum(nnz)), st,
            {k: (v[0] / v[1] if v[1] else None) for k, v in ph.items()})


def fill_bytes(ps, nnz, band_pairs):
    """Algorithmic bytes of one fill launch: 8 per neighbour pair written (int32 col +
    float32 dist), per particle its FP16 record (8), original index (4), fixed-point
    position (8 d), cell key (4) and row bounds (8), and 8 d per FP64 recheck gather."""
    d = ps.dim
    return 8 * nnz + ps.n * (24 + 8 * d) + 8 * d * band_pairs


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the oracle's parallel search uses here: OMP_NUM_THREADS when set (the
    process's CPU share), else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(ps, budget_s=30.0):
    """The oracle as it is, on the same workload, timed on this host: the serial C cell link
    list on one thread (the paper's single-core baseline) and the same arithmetic with rows
    in parallel on every thread of this process's CPU share; median of 3 runs each (fewer if
    the budget runs out)."""
    import oracle

    def timed(fn):
        runs, nnz = [], None
        t_start = time.perf_counter()
        while len(runs) < 3 and (len(runs) == 0 or time.perf_counter() - t_start < budget_s / 2):
            t0 = time.perf_counter()
            rp, _, _ = fn()
            runs.append(time.perf_counter() - t0)
            nnz = int(rp[-1])
        return statistics.median(runs), len(runs), nnz

    threads = host_threads()
    tp, kp, nnz = timed(lambda: oracle.search_par(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, threads=threads))
    t1, k1, nnz1 = timed(lambda: oracle.search_ps(ps))
    assert nnz1 == nnz
    model = cpu_model()
    return {"value": nnz / tp / 1e9, "unit": "Gpairs/s", "cores": threads, "kind": "oracle",
            "sample": f"whole {ps.name} ({ps.n} particles, {nnz} pairs), median of {kp} runs of the C cell "
                      f"link list with rows in parallel on {threads} threads ({tp:.3f} s each)",
            "ms": tp * 1e3, "particles_per_s": ps.n / tp, "cpu_model": model, "nproc": os.cpu_count(),
            "single_thread": {"value": nnz / t1 / 1e9, "unit": "Gpairs/s", "cores": 1, "ms": t1 * 1e3,
                              "runs": k1, "particles_per_s": ps.n / t1}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the SPH-gradient, half-list and all-list legs (profiling runs of the search kernels)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c0", "c1", "c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 relative-coordinate leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-mix leg")
    ap.add_argument("--no-autotune", action="store_true", help="batch workload: keep the default tuning")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 512 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--no-update", action="store_true", help="skip the incremental-update leg")
    ap.add_argument("--no-c1", action="store_true", help="skip the 2D 1M-particle leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the clustered 32-set batch leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_08586_amd import nnps
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "c3":
        return bench_batch(args)
    ps = workload(args.workload)
    log(f"[bench] workload {ps.name} n={ps.n}")
    pos = torch.from_numpy(ps.pos).cuda()
    ctx = nnps.Context(0)

    ms16, nnz, st16, ph16 = time_mode(ctx, pos, ps, nnps.MODE_FP16_RCLL, args.steps, args.warmup)
    log(f"[bench] fp16-rcll {ms16:.3f} ms/step nnz={nnz} phases={ph16}")
    res64 = None
    if not args.no_fp64:
        ms64, nnz64, st64, ph64 = time_mode(ctx, pos, ps, nnps.MODE_FP64_BASELINE, args.steps, args.warmup)
        assert nnz64 == nnz
        log(f"[bench] fp64-baseline {ms64:.3f} ms/step phases={ph64}")
        res64 = {"value": nnz / (ms64 * 1e-3) / 1e9, "unit": "Gpairs/s", "ms_per_step": ms64,
                 "phases_ms": ph64, "speedup_fp16_over_fp64": ms64 / ms16}
    res32 = None
    if not args.no_fp32:
        ms32, nnz32, st32, ph32 = time_mode(ctx, pos, ps, nnps.MODE_FP32_RCLL, args.steps, args.warmup)
        assert nnz32 == nnz
        log(f"[bench] fp32-rcll {ms32:.3f} ms/step phases={ph32}")
        res32 = {"value": nnz / (ms32 * 1e-3) / 1e9, "unit": "Gpairs/s", "ms_per_step": ms32,
                 "phases_ms": ph32, "speedup_fp16_over_fp32": ms32 / ms16,
                 "count_kernel_ms": ph32["count"],
                 "fp32_stats": {"band_pairs": st32["band_pairs"], "false_pos": st32["fp16_false_pos"],
                                "false_neg": st32["fp16_false_neg"]}}
    ctx.close()
    copy_gbs = measured_copy_gbs()
    log(f"[bench] device copy {copy_gbs:.0f} GB/s (read + write)")
    ceil = valu_ceilings()
    log(f"[bench] VALU issue ceilings (wave-instr/s): { {k: f'{v:.3e}' for k, v in ceil.items()} }")
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float32, device="cuda")  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fill_ms = ph16["fill"]
    fb = fill_bytes(ps, nnz, st16["band_pairs"])
    traffic, traffic_detail = fill_traffic() if args.workload == "c2" else (None, None)
    achieved = fb / (fill_ms * 1e-3) / 1e9
    out = {
        "metric": "Gpairs/s at 1M-particle 3D NNPS, FP16 RCLL vs FP64; p50/p99 request latency",
        "value": nnz / (ms16 * 1e-3) / 1e9,
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms16,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": describe(ps),
        "roofline": {"bound": "hbm", "kernel": "k_fill<3,0> (fill pass)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_detail": traffic_detail,
                     "algorithmic_bytes_per_launch": fb, "avg_launch_ms": fill_ms,
                     "measured_copy_gbs": copy_gbs},
        "particles_per_s": ps.n / (ms16 * 1e-3),
        "nnz": nnz,
        "phases_ms": ph16,
        "issue_rate": issue_rates(ph16, ceil) if args.workload == "c2" else None,
        "valu_ceilings": {"unit": "wave64 VALU instructions/s", **ceil,
                          "nominal_one_per_cu_cycle": 256 * 2.4e9},
        "fp16_stats": {k: st16[k] for k in ("candidates", "band_pairs", "fp16_false_pos",
                                              "fp16_false_neg", "heavy_rows", "dense_rows")},
        "fp64_baseline": res64,
        "fp32_rcll": res32,
    }
    if res64 is not None:
        # build + count only (no CSR written), from the per-phase means: isolates the test
        build_count = ("assign", "cellscan", "sort", "pack", "blocks", "unions", "count", "dcount", "rowscan")
        c16 = sum(ph16[k] or 0.0 for k in build_count)
        c64 = sum(ph64[k] or 0.0 for k in build_count)
        out["count_only"] = {"fp16_ms": c16, "fp64_ms": c64, "speedup_fp16_over_fp64": c64 / c16,
                             "count_kernel_speedup": ph64["count"] / ph16["count"],
                             "note": "sum of per-phase means of build + count + row scan; not the headline"}
    if not args.no_update:
        out["update"] = bench_update(ps, pos, args.steps, args.warmup, rebuild_ms=ms16, rebuild_phases=ph16)
    if args.workload == "c2" and not args.no_c1:
        out["c1"] = bench_config("c1", args)
    if args.workload in ("c1", "c2") and not args.no_extras:
        out["sph_gradient"] = bench_gradient(ctx_grad_ps=ps, pos=pos, steps=max(args.steps, 5))
        # half lists (each unordered pair once): the same step with nnps_cells_set_half
        ctx_h = nnps.Context(0)
        msh, nnzh, _, phh = time_batch(ctx_h, [ps], nnps.MODE_FP16_RCLL, args.steps, args.warmup, pos=[pos],
                                       phase_steps=args.steps, half=True)
        ctx_h.close()
        log(f"[bench] half lists {msh:.3f} ms/step nnz={nnzh}")
        out["half_list"] = {"ms_per_step": msh, "nnz": nnzh, "pairs_per_s": nnzh / (msh * 1e-3),
                            "directed_gpairs_per_s": 2 * nnzh / (msh * 1e-3) / 1e9,
                            "count_ms": phh["count"], "fill_ms": phh["fill"]}
    if not args.no_extras:
        out["allpairs_vs_cells"] = bench_allpairs()
    if not args.no_serving:
        out["serving"] = bench_serving(args)
    if args.workload == "c2" and not args.no_c3:
        out["c3"] = bench_batch(args, steps=min(args.steps, 10), warmup=1, sweeps=1, space=C3_SPACE)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(ps)
    print(json.dumps(out), flush=True)


def bench_config(name, args):
    """Another lattice configuration (FP16 RCLL and the FP64 cell list), same step."""
    import torch
    from paper_2401_08586_amd import nnps
    ps = workload(name)
    log(f"[bench] {name}: {ps.name} n={ps.n}")
    pos = torch.from_numpy(ps.pos).cuda()
    ctx = nnps.Context(0)
    steps = min(args.steps, 10)
    ms16, nnz, st16, ph16 = time_mode(ctx, pos, ps, nnps.MODE_FP16_RCLL, steps, args.warmup)
    ms64, nnz64, _, ph64 = time_mode(ctx, pos, ps, nnps.MODE_FP64_BASELINE, steps, args.warmup)
    ctx.close()
    assert nnz64 == nnz
    fb = fill_bytes(ps, nnz, st16["band_pairs"])
    gbs = fb / (ph16["fill"] * 1e-3) / 1e9
    log(f"[bench] {name}: fp16 {ms16:.3f} ms/step, fp64 {ms64:.3f} ms/step, nnz={nnz}")
    del pos
    torch.cuda.empty_cache()
    return {"config": describe(ps), "steps": steps, "value": nnz / (ms16 * 1e-3) / 1e9, "unit": "Gpairs/s",
            "ms_per_step": ms16, "particles_per_s": ps.n / (ms16 * 1e-3), "nnz": nnz, "phases_ms": ph16,
            "fp64_baseline": {"value": nnz / (ms64 * 1e-3) / 1e9, "ms_per_step": ms64, "phases_ms": ph64,
                              "speedup_fp16_over_fp64": ms64 / ms16},
            "fp16_stats": {k: st16[k] for k in ("candidates", "band_pairs", "fp16_false_pos", "fp16_false_neg")},
            "roofline": {"bound": "hbm", "kernel": "k_fill<2,0> (fill pass)", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": fb,
                         "avg_launch_ms": ph16["fill"], "traffic": None}}


def bench_update(ps, pos, steps, warmup, rebuild_ms, rebuild_phases, frac=0.05):
    """Incremental update (nnps_batch_update_step: the displacement applied on the device,
    migrants re-binned, then count and fill) against the full rebuild step. Each step moves
    every particle by the serving mix's motion, U(+-frac dx) per component reflected at the
    box, alternately by +d and -d so the set stays put over many steps; timed as graph
    replays, with per-phase means from as many eager steps."""
    import numpy as np
    import torch
    from paper_2401_08586_amd import nnps
    from paper_2401_08586_amd import workloads as W
    dx = ps.radius / 2.4
    d = W.reflected_displacement(ps.pos, ps.lo, ps.hi, frac * dx, seed=5)
    w = ps.cell_size
    lo = np.asarray(ps.lo)
    migr = float(np.mean(np.any(np.floor((ps.pos + d - lo) / w) != np.floor((ps.pos - lo) / w), axis=1)))
    disp = [torch.from_numpy(d).cuda(), torch.from_numpy(-d).cuda()]
    p = pos.clone()
    ctx = nnps.Context(0)
    cells = ctx.cells()
    cells.build(p, ps.lo, ps.hi, ps.cell_size, ps.radius)
    rp = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
    nnz0 = cells.count(rp)
    cap = int(nnz0 * 1.02) + 4096
    col = torch.empty(cap, dtype=torch.int32, device="cuda")
    dist = torch.empty(cap, dtype=torch.float32, device="cuda")
    cells.fill(rp, col, dist)
    torch.cuda.synchronize()  # the steps below rewrite this structure on another stream
    stream = torch.cuda.Stream()
    cells.set_graphs(True)
    k = 0
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            cells.batch_update_step([rp], [col], [dist], disp=[disp[k % 2]], stream=stream)
            k += 1
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            cells.batch_update_step([rp], [col], [dist], disp=[disp[k % 2]], stream=stream)
            k += 1
        e1.record(stream)
        stream.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nnz = cells.batch_nnz(stream=stream)[0]
    # the same positions searched from scratch give the same count
    c2 = ctx.cells()
    c2.build(p.clone(), ps.lo, ps.hi, ps.cell_size, ps.radius)
    assert c2.count(torch.empty_like(rp)) == nnz
    c2.close()
    cells.set_graphs(False)
    cells.set_profiling(True)
    with torch.cuda.stream(stream):
        for _ in range(steps):
            cells.batch_update_step([rp], [col], [dist], disp=[disp[k % 2]], stream=stream)
            k += 1
    ph = {kk: (v[0] / v[1] if v[1] else None) for kk, v in cells.phase_times(stream=stream).items()}
    cells.close()
    ctx.close()
    build_keys = ("assign", "cellscan", "sort", "pack", "blocks", "unions")
    upd_build = sum(ph[kk] or 0.0 for kk in build_keys)
    reb_build = sum(rebuild_phases[kk] or 0.0 for kk in build_keys)
    log(f"[bench] update step {ms:.3f} ms (rebuild {rebuild_ms:.3f}); structure {upd_build:.3f} ms vs "
        f"{reb_build:.3f} ms; {100 * migr:.1f} % migrate per step")
    return {"ms_per_step": ms, "rebuild_ms_per_step": rebuild_ms, "speedup_over_rebuild": rebuild_ms / ms,
            "value": nnz / (ms * 1e-3) / 1e9, "unit": "Gpairs/s", "nnz": nnz,
            "structure_ms": upd_build, "rebuild_structure_ms": reb_build, "phases_ms": ph,
            "migrating_fraction_per_step": migr,
            "motion": f"U(+-{frac} dx) per component, reflected at the box, alternately +d and -d",
            "note": "update step includes applying the displacement to the binary64 positions; "
                    "the rebuild step's positions are already in place"}


def bench_allpairs(sizes=(1000, 4000, 16000, 64000), reps=20):
    """All-list search (Fig. 3a) against the FP64 and FP16 cell lists on small uniform 3D
    sets, as whole calls (each returns a ready CSR; both read a count back to the host):
    mean wall time per call over `reps` calls after one warm-up call."""
    import torch
    from paper_2401_08586_amd import nnps
    from paper_2401_08586_amd import workloads as W
    ctx = nnps.Context(0)
    out = []
    for n in sizes:
        ps = W.uniform(3, n, seed=n)
        pos = torch.from_numpy(ps.pos).cuda()
        row = {"n": n}
        c64, c16 = ctx.cells(), ctx.cells()  # cell structures reused across calls
        calls = {
            "allpairs_ms": lambda: nnps.allpairs_search(pos, ps.lo, ps.hi, ps.radius, ctx=ctx),
            "cells_fp64_ms": lambda: nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius,
                                                 mode=nnps.MODE_FP64_BASELINE, ctx=ctx, cells=c64),
            "cells_fp16_ms": lambda: nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, ctx=ctx,
                                                 cells=c16),
        }
        for name, call in calls.items():
            r = call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = call()
            torch.cuda.synchronize()
            row[name] = (time.perf_counter() - t0) * 1e3 / reps
            if name == "allpairs_ms":
                row["nnz"] = int(r[1].numel())
            else:
                assert int(r[1].numel()) == row["nnz"]
        c64.close()
        c16.close()
        log(f"[bench] allpairs vs cells {row}")
        out.append(row)
    ctx.close()
    return out


def bench_gradient(ctx_grad_ps, pos, steps):
    """The SPH gradient (Eq. 2 and Eq. A5) of f = x^3 over this workload's neighbour list:
    mean kernel time over `steps` launches (HIP events on the launch stream) and its HBM
    roofline with algorithmic bytes 4 per pair (column index) plus, per particle, position
    8d, field 8, row bounds 8 and both outputs 16d."""
    import torch
    from paper_2401_08586_amd import nnps
    ps = ctx_grad_ps
    ctx = nnps.Context(0)
    rp, col, _, cells = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, ctx=ctx)
    nnz = int(col.numel())
    f = (pos[:, 0] ** 3).contiguous()
    h = ps.radius / 2.0
    torch.cuda.synchronize()  # the list is written on the null stream, read on another
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        nnps.sph_gradient(pos, f, h, rp, col, ctx=ctx, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            nnps.sph_gradient(pos, f, h, rp, col, ctx=ctx, stream=stream)
        e1.record(stream)
    stream.synchronize()
    ms = e0.elapsed_time(e1) / steps
    d = ps.dim
    nbytes = 4 * nnz + ps.n * (8 * d + 8 + 8 + 16 * d)
    gbs = nbytes / (ms * 1e-3) / 1e9
    ctx.close()
    log(f"[bench] sph gradient {ms:.3f} ms ({nnz / (ms * 1e-3) / 1e9:.1f} Gpairs/s)")
    return {"ms": ms, "gpairs_per_s": nnz / (ms * 1e-3) / 1e9, "dtype": "f64",
            "roofline": {"bound": "hbm", "kernel": "k_sph_gradient", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": nbytes}}


def serving_leg(sims, args, slots, load, **kw):
    """Saturated rate closed-loop, then Poisson arrivals at `load` times it."""
    from paper_2401_08586_amd import serving as S
    nsims = len(sims)
    srv = S.Server(sims, slots=slots, **kw)
    sat = srv.run([], closed_loop=5 * nsims)
    cal = S.summarize(sat, warmup=nsims)
    rate = load * cal["requests_per_s"]
    warm = max(args.serving_requests // 10, nsims)
    arrivals = S.poisson_arrivals(rate, args.serving_requests + warm, nsims, seed=11)
    done = srv.run(arrivals)
    res = S.summarize(done, warmup=warm)
    res.update(srv.counters())
    srv.close()
    res.update({"saturated_requests_per_s": cal["requests_per_s"], "saturated_gpairs_per_s": cal["gpairs_per_s"],
                "arrival_rate_per_s": rate, "load": load, "warmup_requests": warm, "slots": slots})
    return res


def bench_serving(args, nsims=64, slots=4, load=0.7):
    """Serving mix: 64 simulations (half 2D, half 3D lattices, 1e3..2e6 particles), each
    request one time step (move by U(+-0.05 dx) reflected at the box, update the resident
    structure, search). Latency = arrival to CSR ready (device event). Legs: the default
    (incremental updates, admission by free HBM), the same with a byte budget of 60 % of
    the mix's footprint (forces admissions and evictions), full rebuilds instead of
    updates, and requests batched per slot (one batch call per slot, rebuilt)."""
    import torch
    from paper_2401_08586_amd import serving as S
    from paper_2401_08586_amd import workloads as W
    sims = W.serving_sims(nsims)
    log(f"[bench] serving: {nsims} sims, {sum(p.n for p in sims)} particles")
    res = serving_leg(sims, args, slots, load)
    log(f"[bench] serving (update): p50 {res['p50_ms']:.3f} ms p99 {res['p99_ms']:.3f} ms "
        f"{res['gpairs_per_s']:.2f} Gpairs/s; tail queue {res['tail_queue_ms']:.3f} ms device "
        f"{res['tail_device_ms']:.3f} ms")
    # the mix's resident footprint as the server estimates it (positions and displacements,
    # CSR at 1.1x the expected neighbours, a cell structure per simulation)
    total = sum(p.n * p.dim * 16 + (p.n + 1) * 8 + int(p.n * (20 if p.dim == 2 else 60) * 1.1 * 8) + 4096 * 8
                + p.n * (200 + 16 * 3 ** p.dim) for p in sims)
    legs = {}
    for name, kw in (("budget_60pct", {"budget_bytes": 0.6 * total}), ("rebuild", {"use_update": False}),
                     ("batched", {"per_sim": False})):
        r = serving_leg(sims, args, slots, load, **kw)
        log(f"[bench] serving ({name}): p50 {r['p50_ms']:.3f} ms p99 {r['p99_ms']:.3f} ms "
            f"{r['gpairs_per_s']:.2f} Gpairs/s mean batch {r['mean_batch']:.1f} admissions {r['admissions']} "
            f"evictions {r['evictions']}")
        legs[name] = {k: r[k] for k in ("p50_ms", "p99_ms", "gpairs_per_s", "requests_per_s", "mean_batch",
                                         "admissions", "evictions", "budget_bytes", "saturated_requests_per_s",
                                         "queue_p99_ms", "device_p99_ms", "tail_queue_ms", "tail_device_ms")}
        torch.cuda.empty_cache()
    res.update({"sims": nsims, "particles": sum(p.n for p in sims), "footprint_bytes_estimate": total,
                "workload": "64 jittered lattices (32 2D, 32 3D), n log-uniform 1e3..2e6, per-step move "
                            "U(+-0.05 dx) reflected at the box faces, Poisson arrivals",
                "legs": legs})
    return res


# a smaller search space for the clustered batch inside the default run (about ten settings)
C3_SPACE = {"block_target": [48, 64, 80, 96], "dense_min_union": [256, 512, 1024], "dense_grid": [1024, 1280, 2048]}


def bench_batch(args, steps=None, warmup=None, sweeps=2, space=None):
    """32 clustered 3D sets (sizes log-uniform in [1e4, 1e6]) searched as one batch, with the
    work shapes picked by the autotuner first (coordinate descent, `sweeps` passes)."""
    import torch
    from paper_2401_08586_amd import nnps
    from paper_2401_08586_amd import workloads as W
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    pss = W.clustered_batch()
    ntot = sum(p.n for p in pss)
    log(f"[bench] batch of {len(pss)} clustered sets, {ntot} particles")
    ctx = nnps.Context(0)
    tuned = None
    if not args.no_autotune:
        from paper_2401_08586_amd import autotune as A
        sets = [(torch.from_numpy(p.pos).cuda(), p.lo, p.hi, p.cell_size, p.radius) for p in pss]
        t0 = time.perf_counter()
        best, best_ms, evals = A.tune(ctx, sets, pss, nnps.MODE_FP16_RCLL, use_cache=False, log=log, sweeps=sweeps,
                                      space=space)
        tuned = {"params": best, "ms_per_step_at_tuning": best_ms, "evaluations": evals,
                 "tuning_s": time.perf_counter() - t0, "sweeps": sweeps, "space": space or A.SPACE}
        del sets
        torch.cuda.empty_cache()
        log(f"[bench] autotuned {best} ({evals} settings, {tuned['tuning_s']:.1f} s)")
    ms, nnz, st, ph = time_batch(ctx, pss, nnps.MODE_FP16_RCLL, steps, warmup)
    log(f"[bench] batch fp16-rcll {ms:.3f} ms/step nnz={nnz} phases={ph}")
    ctx.close()
    torch.cuda.empty_cache()
    # the fill passes (block, long-row and dense-cell) together write the CSR: 8 bytes per
    # pair, plus per particle its row bounds (8) and one read of its FP16 record and
    # original index (12); the dense-cell fill writes most of it
    fill_ms = sum(ph[k] or 0.0 for k in ("fill", "longrows", "dfill"))
    fb = 8 * nnz + 20 * ntot
    out = {
        "metric": "Gpairs/s, batched clustered 3D NNPS (32 sets, FP16 RCLL)",
        "value": nnz / (ms * 1e-3) / 1e9, "unit": "Gpairs/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "clustered_batch_32", "sets": len(pss), "particles": ntot,
                   "sizes": sorted(p.n for p in pss)},
        "nnz": nnz, "particles_per_s": ntot / (ms * 1e-3), "phases_ms": ph,
        "fp16_stats": {k: st[k] for k in ("candidates", "band_pairs", "fp16_false_pos", "fp16_false_neg",
                                          "heavy_rows", "dense_rows", "dense_entries")},
        "autotune": tuned,
        "roofline": {
            "bound": "hbm", "kernel": "fill passes (k_fill<3,0>, k_long, k_dense<3,0,true,*>)",
            "achieved": fb / (fill_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": fb / (fill_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": fb,
            "avg_launch_ms": fill_ms, "traffic": None},
    }
    if args.workload == "c3":
        print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
