"""The serving loop on the GPU: continuous batching over two stream slots with a memory
budget small enough to force evictions. Every result is the same as the same step's
search alone (bit for bit), whatever the schedule: a second run with one slot and no
budget reproduces every (simulation, step) exactly, and sampled steps match the oracle."""
import numpy as np
import pytest

import oracle
from paper_2401_08586_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2401_08586_amd import nnps  # noqa: E402
from paper_2401_08586_amd import serving as S  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nnps.Context(0)
    yield c
    c.close()


def serve(ctx, sims, slots, budget, arrivals, per_sim=True):
    srv = S.Server(sims, slots=slots, budget_bytes=budget, max_batch_particles=60000, ctx=ctx, keep_results=True,
                   per_sim=per_sim)
    done = srv.run(arrivals)
    out = dict(srv.results)
    ev = srv.sched.evictions
    nb = srv.batches
    srv.close()
    return done, out, ev, nb


@pytest.mark.parametrize("per_sim", [True, False], ids=["per_sim_graphs", "batched"])
def test_serving_results_equal_alone_and_in_the_mix(ctx, per_sim):
    sims = W.serving_sims(8, seed=7, lo=1e3, hi=5e4)
    total = sum(p.n * p.dim * 8 + (p.n + 1) * 8 + p.n * 60 * 8 + (p.n * (200 + 16 * 3 ** p.dim) if per_sim else 0)
                for p in sims)
    arrivals = S.poisson_arrivals(3000.0, 60, nsims=len(sims), seed=9)
    print(f"[gpu] serving {len(sims)} sims, {sum(p.n for p in sims)} particles, per_sim={per_sim}", flush=True)
    done, res, evictions, batches = serve(ctx, sims, 2, total * 0.4, arrivals, per_sim)
    assert len(done) == 60 and len(res) == 60
    assert evictions > 0, "the budget should force evictions"
    if not per_sim:
        assert batches < 60, "requests should share batches"
    assert all(r.latency_ms > 0 for r in done)
    cells = ctx.cells()
    for (s, step), (pos, rp, col, dist) in sorted(res.items()):
        ps = sims[s]
        arp, acol, adist, _ = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, ctx=ctx, cells=cells)
        assert torch.equal(arp, rp) and torch.equal(acol, col) and torch.equal(adist, dist), (s, step)
    cells.close()
    # a different schedule (one slot, no budget) gives the same (sim, step) results
    print("[gpu] serving again, one slot", flush=True)
    done2, res2, ev2, _ = serve(ctx, sims, 1, float("inf"), arrivals, per_sim)
    assert ev2 == 0 and res2.keys() == res.keys()
    for key in res:
        for a, b in zip(res[key], res2[key]):
            assert torch.equal(a, b), key
    # sampled steps against the oracle
    for key in sorted(res)[::7]:
        s, _ = key
        ps = sims[s]
        pos, rp, col, dist = (t.cpu().numpy() for t in res[key])
        wrp, wcol, wdist = oracle.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius)
        np.testing.assert_array_equal(rp, wrp)
        np.testing.assert_array_equal(col, wcol)
        assert np.all(np.abs(dist - wdist.astype(np.float64)) <= 1e-6 * wdist.astype(np.float64))


def test_serving_closed_loop(ctx):
    sims = W.serving_sims(6, seed=8, lo=1e3, hi=2e4)
    srv = S.Server(sims, slots=2, ctx=ctx)
    done = srv.run([], closed_loop=40)
    srv.close()
    assert len(done) == 40
    steps = {}
    for r in done:
        steps.setdefault(r.sim, []).append(r.step)
    for s, st in steps.items():
        assert sorted(st) == list(range(len(st))), (s, st)  # each sim's steps in order, none lost
    out = S.summarize(done)
    assert out["p99_ms"] >= out["p50_ms"] > 0
