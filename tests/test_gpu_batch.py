"""Batched modeling of jobs with different grids (fwime_model_batch).

Each job's data must match the FP64 oracle for that job (relative L2 <= 1e-4)
and equal what fwime_model computes for that job alone, bit for bit (the
per-cell arithmetic does not depend on the launch), with and without the
captured graph, across graph replays interleaved with eager work, and for
whichever tile width the autotuner picks.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from _helpers import gpu_problem, oracle_problem_f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_02362_amd as fw
    c = fw.Context(0)
    yield c
    c.close()


def _jobs_small():
    a = synth.tiny(nz=30, nx=50, nb=8, nt=120, nshots=2, seed=1)
    b = synth.tiny(nz=50, nx=70, nb=10, nt=200, nshots=3, seed=2)
    c = synth.tiny(nz=40, nx=90, nb=6, nt=90, nshots=1, seed=3)
    return [a, b, c]


def _run_single(ctx, ws):
    outs = []
    for w in ws:
        grid, tv, tg = gpu_problem(w)
        outs.append(ctx.model(grid, tv, tg).cpu().numpy())
    return outs


def _run_batch(ctx, ws):
    probs = [gpu_problem(w) for w in ws]
    outs = ctx.model_batch(probs)
    return [o.cpu().numpy() for o in outs]


def test_batch_equals_single_calls(ctx):
    say("case: batch of 3 uneven jobs vs single calls")
    ws = _jobs_small()
    ref = _run_single(ctx, ws)
    info0 = ctx.info()
    out = _run_batch(ctx, ws)
    info1 = ctx.info()
    for r, o in zip(ref, out):
        assert np.array_equal(r, o)
    assert info1["last_batch_tile_x"] in (16, 24, 32, 48, 64)
    assert info1["tuned_signatures"] == info0["tuned_signatures"] + 1
    # same shapes again: the tuned width is reused, not re-tuned
    out2 = _run_batch(ctx, ws)
    assert ctx.info()["tuned_signatures"] == info1["tuned_signatures"]
    for r, o in zip(ref, out2):
        assert np.array_equal(r, o)


def test_batch_matches_oracle(ctx):
    # every job of an uneven batch (three grids, 1-3 shots, different nt and
    # strips) against the FP64 oracle, on the direct-launch path and on the
    # graph path
    import torch
    say("case: batch of 3 uneven jobs vs oracle.model")
    ws = _jobs_small()
    refs = []
    for w in ws:
        g, geo, vel = oracle_problem_f32(w)
        refs.append(oracle.model(g, vel, geo))
    old = os.environ.pop("FWIME_NO_GRAPH", None)
    try:
        for no_graph in ("1", None):
            if no_graph:
                os.environ["FWIME_NO_GRAPH"] = no_graph
            else:
                os.environ.pop("FWIME_NO_GRAPH", None)
            out = _run_batch(ctx, ws)
            torch.cuda.synchronize()
            for w, r, o in zip(ws, refs, out):
                e = rel_l2(o, r)
                say(f"  {w.name} nt {w.nt} shots {w.nshots} graph {no_graph is None}: rel-L2 {e:.3e}")
                assert e < 1e-4
    finally:
        if old is not None:
            os.environ["FWIME_NO_GRAPH"] = old
        else:
            os.environ.pop("FWIME_NO_GRAPH", None)


def test_batch_graph_replays_with_eager_work_between(ctx):
    import torch
    say("case: graph replays interleaved with eager calls")
    ws = _jobs_small()
    old = os.environ.pop("FWIME_NO_GRAPH", None)
    try:
        os.environ["FWIME_NO_GRAPH"] = "1"
        eager = _run_batch(ctx, ws)
        del os.environ["FWIME_NO_GRAPH"]
        for k in range(3):
            out = _run_batch(ctx, ws)            # graph path (replayed several times per call)
            _run_single(ctx, ws[:1])             # eager work in between
            torch.cuda.synchronize()
            for e, o in zip(eager, out):
                assert np.array_equal(e, o), k
    finally:
        if old is not None:
            os.environ["FWIME_NO_GRAPH"] = old
        else:
            os.environ.pop("FWIME_NO_GRAPH", None)


def test_batch_full_size_grids(ctx):
    say("case: batch on 200x600, 300x1700, 500x2500 grids, nt 300")
    ws = synth.batch_set(nshots=6, seed=7, nt_range=(250, 300))
    ref = _run_single(ctx, ws)
    out = _run_batch(ctx, ws)
    for r, o in zip(ref, out):
        assert np.array_equal(r, o)
