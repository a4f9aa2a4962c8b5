"""The allocation-free modeling entry point (fwime_model_static) through the C ABI.

Its scratch is the library's static device array instead of the context's
arena.  Two calls in a row, the second with a smaller input, must each equal
fwime_model's output bit for bit (same kernels, same per-cell arithmetic);
the array keeps the previous call's contents, so this also checks that the
call clears what must start at zero.  A call whose single shot does not fit
the array is rejected with FWIME_ENOMEM and leaves its output untouched, and
the call grows no arena.
"""
import sys

import numpy as np
import pytest

import synth
from _helpers import gpu_problem

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _static_vs_arena(ctx, w):
    import torch
    grid, tv, tg = gpu_problem(w)
    ref = ctx.model(grid, tv, tg)
    out = torch.full((w.nshots, w.nrec, w.nt), 3.0, device="cuda:0")
    arena_before = ctx.info()["arena_bytes"]
    ctx.fwime_model_static(grid, tv, tg, out)
    torch.cuda.synchronize()
    assert ctx.info()["arena_bytes"] == arena_before
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_model_equals_model_twice_second_smaller():
    import paper_2206_02362_amd as fw
    ctx = fw.Context(0)
    # first call: the 300 x 1700 Marmousi-like grid (60-cell strip), 10 shots,
    # nt 400: 13 MB of wavefields per shot, so the 64 MiB array runs the
    # shots in three batches (fwime_model runs them in one)
    w1 = synth.marmousi_set(10, 170)
    w1.nt = 400
    w1.wavelet = w1.wavelet[:, :400].copy()
    say("case: static-scratch modeling, 300x1700 nb60 nt400 10 shots")
    ref, out = _static_vs_arena(ctx, w1)
    assert np.abs(ref).max() > 0 and np.array_equal(ref, out)
    # second call: smaller grid, fewer shots and steps, over the first
    # call's leftovers in the array
    w2 = synth.tiny(nz=30, nx=44, nb=6, nt=90, nshots=2, seed=4)
    say("case: static-scratch modeling, 30x44 nb6 nt90 2 shots")
    ref, out = _static_vs_arena(ctx, w2)
    assert np.abs(ref).max() > 0 and np.array_equal(ref, out)
    ctx.close()


def test_static_model_rejects_a_shot_beyond_the_array():
    import torch
    import paper_2206_02362_amd as fw
    ctx = fw.Context(0)
    # one shot's four wavefields on 1500 x 3000 (+ 2 x 40 strip) cells are
    # about 80 MB, beyond the 64 MiB array
    say("case: static-scratch modeling, 1500x3000 one shot: rejected")
    nz, nx, nt = 1500, 3000, 20
    grid = fw.Grid(nz, nx, 40, nt, 10.0, 10.0, 1e-3)
    vel = torch.full((nx, nz), 2000.0, device="cuda:0")
    geo = fw.Geometry(np.array([2], np.int32), np.array([10], np.int32), np.full((1, 4), 2, np.int32),
                      np.arange(4, dtype=np.int32)[None], torch.ones((1, nt), device="cuda:0"))
    data = torch.full((1, 4, nt), 7.0, device="cuda:0")
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_model_static(grid, vel, geo, data)
    assert e.value.code == fw.FWIME_ENOMEM
    torch.cuda.synchronize()
    assert bool(torch.all(data == 7.0))
    ctx.close()
