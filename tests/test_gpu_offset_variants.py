"""Alternative offset kernels against the defaults, bit for bit.

The scatter / spread exists as the LDS ring fed by 16-byte direct loads (the
default) and as the register-staged ring (FWIME_SCATTER_KERNEL=ws); the
wide-offset imaging condition as the direct-load ring (the default) and the
register-staged ring (FWIME_IMAGE_KERNEL=lds).  Each pair forms the same
products and sums them in the same order, so extended Born data, adjoint
images and gradients must agree bit for bit.  nh = 61 (H = 30, the widest
kernels), 21 and 5, on a grid whose width is not a multiple of the scatter's
48-column blocks and whose strips start above the model (the direct-load
kernels align them to 64-byte boundaries, the register-staged ones do not).
"""
import sys

import numpy as np
import pytest

import synth
from _helpers import gpu_problem

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# 70 rows: the direct-load strips start 8 rows above the model (2 strips
# either way); 60 rows: starting them there would take a second strip, so
# they start at the model's first row
@pytest.mark.parametrize("nz", [70, 60])
@pytest.mark.parametrize("nh", [61, 21, 5])
def test_offset_kernel_variants_bitwise(nh, nz, monkeypatch):
    import torch
    import paper_2206_02362_amd as fw
    say(f"case: offset kernel variants, {nz}x150 nb8 nt121, 2 shots, nh {nh}")
    w = synth.tiny(nz=nz, nx=150, nb=8, nt=121, nshots=2, nh=nh, seed=7)
    grid, tv, tg = gpu_problem(w)
    pt = torch.tensor(1e-2 * synth.random_ptilde(nh, w.nz, w.nx, 3), dtype=torch.float32, device="cuda:0")
    dobs = torch.tensor(1e-3 * np.random.default_rng(5).standard_normal((w.nshots, w.nrec, w.nt)),
                        dtype=torch.float32, device="cuda:0")
    dso = synth.dso_weights(nh)
    ctx = fw.Context(0)

    def run():
        born = ctx.born_ext_fwd(grid, tv, tg, pt).cpu().numpy()
        adj = ctx.born_ext_adj(grid, tv, tg, dobs, nh).cpu().numpy()
        _, gv, gp = ctx.gradient(grid, tv, tg, pt, dobs, 1e-3, dso)
        torch.cuda.synchronize()
        return born, adj, gv.cpu().numpy(), gp.cpu().numpy()

    names = ("born_fwd", "born_adj", "grad_vel", "grad_ptilde")
    ref = run()
    monkeypatch.setenv("FWIME_SCATTER_KERNEL", "ws")
    monkeypatch.setenv("FWIME_IMAGE_KERNEL", "lds")
    alt = run()
    ctx.close()
    for name, a, b in zip(names, ref, alt):
        say(f"  {name}: max |x| {np.abs(a).max():.3e}, max |diff| {np.abs(a - b).max():.3e}")
        assert np.abs(a).max() > 0, name
        assert np.array_equal(a, b), name
