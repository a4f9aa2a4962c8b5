"""Two time steps per launch against one step per launch.

The two-step stencil recomputes the intermediate field on a halo and keeps
it in LDS; the arithmetic per cell is the one-step kernel's, so modeled data
and gradients must agree bit for bit (FWIME_STEP1=1 selects one step per
launch when a context is created).  The extended Born pair differs on
purpose: with two steps per launch its background field is carried in
extended precision.  Sources and receivers sit on and next to the 56-row
and TX-column tile boundaries, nt is odd and even, and every tile width is
covered.
"""
import os
import sys

import numpy as np
import pytest

import synth
from _helpers import gpu_problem

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _ctx(step1: bool, tile_x: int):
    import paper_2206_02362_amd as fw
    old = {k: os.environ.get(k) for k in ("FWIME_STEP1", "FWIME_TILE_X")}
    try:
        os.environ["FWIME_TILE_X"] = str(tile_x)
        if step1:
            os.environ["FWIME_STEP1"] = "1"
        else:
            os.environ.pop("FWIME_STEP1", None)
        return fw.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _boundary_workload(nt, tile_x, seed):
    # padded 128 x 150: three 56-row tiles, several x tiles; nb = 6
    nz, nx, nb = 116, 138, 6
    w = synth.tiny(nz=nz, nx=nx, nb=nb, nt=nt, nshots=6, seed=seed, f_peak=20.0, vmax=3000.0)
    # sources on / around row 56 and 112 (padded) and column multiples of tile_x
    pz = [55, 56, 57, 111, 112, 3]
    px = [tile_x - 1, tile_x, 2 * tile_x + 3, 1, 3 * tile_x - 4, nx + 2 * nb - 1]
    w.src_iz = np.array([min(max(z - nb, 0), nz - 1) for z in pz], dtype=np.int32)
    w.src_ix = np.array([min(max(x - nb, 0), nx - 1) for x in px], dtype=np.int32)
    # receivers at several depths crossing tile rows, every 3rd column
    rx = np.arange(0, nx, 3, dtype=np.int32)
    rz = np.array([(50 + 7 * i) % nz for i in range(rx.size)], dtype=np.int32)
    w.rec_ix = np.tile(rx, (6, 1))
    w.rec_iz = np.tile(rz, (6, 1))
    return w


@pytest.mark.parametrize("tile_x", [16, 24, 32, 48, 64])
@pytest.mark.parametrize("nt", [201, 202])
def test_two_step_model_bitwise(tile_x, nt):
    say(f"case: two-step vs one-step model, TX {tile_x}, nt {nt}")
    w = _boundary_workload(nt, tile_x, seed=tile_x + nt)
    grid, tv, tg = gpu_problem(w)
    c1 = _ctx(True, tile_x)
    c2 = _ctx(False, tile_x)
    d1 = c1.model(grid, tv, tg).cpu().numpy()
    d2 = c2.model(grid, tv, tg).cpu().numpy()
    c1.close()
    c2.close()
    assert np.abs(d1).max() > 0
    diff = np.abs(d1 - d2).max()
    say(f"  max |diff| {diff:.3e} (max |d| {np.abs(d1).max():.3e})")
    assert np.array_equal(d1, d2)


@pytest.mark.parametrize("nt", [151, 152])
def test_two_step_born_and_gradient_bitwise(nt):
    import torch
    say(f"case: two-step vs one-step born_fwd / born_adj / gradient, nt {nt}")
    w = _boundary_workload(nt, 32, seed=nt)
    grid, tv, tg = gpu_problem(w)
    nh = 5
    pt = torch.tensor(1e-2 * synth.random_ptilde(nh, w.nz, w.nx, 3), dtype=torch.float32, device="cuda:0")
    dobs = torch.tensor(1e-3 * np.random.default_rng(4).standard_normal((w.nshots, w.nrec, nt)),
                        dtype=torch.float32, device="cuda:0")
    dso = synth.dso_weights(nh)
    outs = []
    for step1 in (True, False):
        c = _ctx(step1, 32)
        born = c.born_ext_fwd(grid, tv, tg, pt).cpu().numpy()
        adj = c.born_ext_adj(grid, tv, tg, dobs, nh).cpu().numpy()
        obj, gv, gp = c.gradient(grid, tv, tg, pt, dobs, 1e-3, dso)
        outs.append((born, adj, obj.cpu().numpy(), gv.cpu().numpy(), gp.cpu().numpy()))
        c.close()
    for name, a, b in zip(("born_fwd", "born_adj", "obj", "grad_vel", "grad_ptilde"), outs[0], outs[1]):
        say(f"  {name}: max |diff| {np.abs(a - b).max():.3e} (max |x| {np.abs(a).max():.3e})")
        assert np.abs(a).max() > 0
        if name.startswith("born"):
            # the two-step path carries the Born background in extended
            # precision (FP32 + BF16 residual): close, not identical
            e = np.linalg.norm(a - b) / np.linalg.norm(a)
            say(f"    rel-L2 one-step vs two-step {e:.3e}")
            assert e < 1e-4, name
        else:
            assert np.array_equal(a, b), name


def test_two_step_batch_matches_one_step_singles():
    say("case: two-step multi-job batch vs one-step single calls (odd and even nt)")
    ws = [synth.tiny(nz=30, nx=50, nb=8, nt=121, nshots=2, seed=1),
          synth.tiny(nz=50, nx=70, nb=10, nt=200, nshots=3, seed=2),
          synth.tiny(nz=40, nx=90, nb=6, nt=91, nshots=1, seed=3)]
    probs = [gpu_problem(w) for w in ws]
    c1 = _ctx(True, 32)
    ref = [c1.model(g, v, ge).cpu().numpy() for g, v, ge in probs]
    c1.close()
    c2 = _ctx(False, 32)
    out = [o.cpu().numpy() for o in c2.model_batch(probs)]
    c2.close()
    for r, o in zip(ref, out):
        assert np.array_equal(r, o)
