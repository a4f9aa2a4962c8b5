"""Continuous batching of modeling jobs (fwime_engine_*) on the GPU.

Jobs of different grids, shot counts and lengths join the engine's running
time loop at different round boundaries and leave when done.  Each job's data
must equal what fwime_model computes for it alone, bit for bit (the per-cell
arithmetic does not depend on which jobs share a launch or on the time index
at which a job joins), and match the FP64 oracle to 1e-4 relative L2.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from _helpers import gpu_problem, oracle_problem_f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _drain(eng, tickets, max_rounds=10000):
    done = set()
    for _ in range(max_rounds):
        done.update(eng.poll())
        if tickets <= done:
            return
        if eng.info()["active"] or eng.info()["pending"]:
            eng.run()
        else:
            eng.stream.synchronize()
    raise AssertionError("engine did not finish its jobs")


def test_engine_jobs_joining_at_different_rounds():
    import torch
    import paper_2206_02362_amd as fw
    say("case: engine, 4 jobs joining at rounds 0, 0, 1 and 3 (8 steps per round)")
    ws = [synth.tiny(nz=30, nx=50, nb=8, nt=120, nshots=2, seed=1),
          synth.tiny(nz=50, nx=70, nb=10, nt=61, nshots=3, seed=2),
          synth.tiny(nz=40, nx=90, nb=6, nt=91, nshots=1, seed=3),
          synth.tiny(nz=26, nx=34, nb=5, nt=40, nshots=2, seed=4)]
    ws[3].src_iz[:] = 1
    probs = [gpu_problem(w) for w in ws]
    probs[3][0].free_surface = True          # a free-surface job in the same launches
    ctx = fw.Context(0)
    ref = [ctx.model(g, v, ge).cpu().numpy() for g, v, ge in probs]
    eng_stream = torch.cuda.Stream()
    check = torch.cuda.current_stream()
    eng = fw.Engine(ctx, eng_stream, steps_per_round=8, max_jobs=8)
    outs = [torch.full((w.nshots, w.nrec, w.nt), 5.0, device="cuda:0") for w in ws]
    tickets = {}
    for k in (0, 1):
        tickets[k] = eng.submit(*probs[k], outs[k], check)
    eng.run()                                 # round 0: jobs 0 and 1
    tickets[2] = eng.submit(*probs[2], outs[2], check)
    eng.run()                                 # round 1: job 2 joins
    eng.run()
    tickets[3] = eng.submit(*probs[3], outs[3], check)
    _drain(eng, set(tickets.values()))
    inf = eng.info()
    say(f"  rounds {inf['rounds']}, launches {inf['launches']}, step {inf['step']}")
    assert inf["active"] == 0 and inf["pending"] == 0 and inf["finishing"] == 0
    for k, (w, r) in enumerate(zip(ws, ref)):
        o = outs[k].cpu().numpy()
        assert np.abs(r).max() > 0
        assert np.array_equal(o, r), k
        g, geo, vel = oracle_problem_f32(w)
        g.free_surface = probs[k][0].free_surface
        e = rel_l2(o, oracle.model(g, vel, geo))
        say(f"  job {k}: nt {w.nt} shots {w.nshots} joined bitwise, oracle rel-L2 {e:.3e}")
        assert e < 1e-4
    eng.close()
    ctx.close()


def test_engine_full_size_grids():
    import torch
    import paper_2206_02362_amd as fw
    say("case: engine, 200x600 / 300x1700 / 500x2500 jobs, nt 200-300, staggered")
    ws = synth.batch_set(nshots=5, seed=9, nt_range=(200, 300))
    probs = [gpu_problem(w) for w in ws]
    ctx = fw.Context(0)
    ref = [ctx.model(g, v, ge).cpu().numpy() for g, v, ge in probs]
    eng = fw.Engine(ctx, torch.cuda.Stream(), steps_per_round=64, max_jobs=8)
    outs = [torch.empty((w.nshots, w.nrec, w.nt), device="cuda:0") for w in ws]
    tickets = set()
    for k, (p, o) in enumerate(zip(probs, outs)):
        tickets.add(eng.submit(*p, o, torch.cuda.current_stream()))
        eng.run()
    _drain(eng, tickets)
    for r, o in zip(ref, outs):
        assert np.array_equal(r, o.cpu().numpy())
    eng.close()
    ctx.close()


def test_engine_rejects_bad_jobs_and_too_many():
    import torch
    import paper_2206_02362_amd as fw
    ctx = fw.Context(0)
    eng = fw.Engine(ctx, torch.cuda.Stream(), steps_per_round=8, max_jobs=1)
    w = synth.tiny(nz=16, nx=20, nb=4, nt=50, nshots=1)
    grid, tv, tg = gpu_problem(w)
    bad = fw.Grid(grid.nz, grid.nx, grid.nb, grid.nt, grid.dz, grid.dx, 0.01)     # CFL violated
    out = torch.empty((1, w.nrec, w.nt), device="cuda:0")
    with pytest.raises(fw.FwimeError) as e:
        eng.submit(bad, tv, tg, out, torch.cuda.current_stream())
    assert e.value.code == fw.FWIME_EINVAL
    t = eng.submit(grid, tv, tg, out, torch.cuda.current_stream())
    with pytest.raises(fw.FwimeError) as e:
        eng.submit(grid, tv, tg, torch.empty_like(out), torch.cuda.current_stream())
    assert e.value.code == fw.FWIME_ENOMEM
    _drain(eng, {t})
    assert np.array_equal(out.cpu().numpy(), ctx.model(grid, tv, tg).cpu().numpy())
    eng.close()
    ctx.close()
