"""torch.autograd path (fwime_forward_tape / fwime_backward_tape).

* parity: the gradient of L = 1/2 ||d_pred - d_obs||^2 through FwimeOp equals the
  FP64 oracle's FWIME gradient at eps = 0 (relative L2 <= 1e-4);
* finite differences on the full 300 x 1700 grid, 50 shots, nt = 5000: central
  differences of L along 10 seeded smooth perturbations of amplitude 1e-3 v
  against <grad, dm> (FP32 loss evaluations, tolerance 1e-2);
* the tape serves one backward and its memory is released.
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


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_02362_amd as fw
    c = fw.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def _autograd_vs_oracle(ctx, w, seed):
    import torch
    import paper_2206_02362_amd as fw
    g, geo, vel = oracle_problem_f32(w)
    true = vel + 120.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 41 + seed, 80.0)
    dobs = oracle.model(g, true, geo).astype(np.float32)
    pt = (0.2 * np.random.default_rng(5 + seed).standard_normal((w.nh, w.nx, w.nz))).astype(np.float32)
    obj_r, gv_r, gp_r = oracle.gradient(g, vel, geo, pt.astype(np.float64), dobs.astype(np.float64), 0.0,
                                        np.ones(w.nh))
    grid, tv, tg = gpu_problem(w)
    v = tv.clone().requires_grad_(True)
    p = _dev(pt).requires_grad_(True)
    d = fw.predicted_data(v, p, ctx, grid, tg)
    loss = 0.5 * ((d.double() - _dev(dobs).double()) ** 2).sum()
    loss.backward()
    e_obj = abs(loss.item() - obj_r) / obj_r
    e_gv = rel_l2(v.grad.double().cpu().numpy(), gv_r)
    e_gp = rel_l2(p.grad.double().cpu().numpy(), gp_r)
    say("  obj", e_obj, "grad_vel", e_gv, "grad_ptilde", e_gp)
    assert e_obj < 1e-4 and e_gv < 1e-4 and e_gp < 1e-4


def test_autograd_matches_oracle_gradient(ctx):
    say("case: autograd vs oracle, tiny nh5")
    _autograd_vs_oracle(ctx, synth.tiny(nz=24, nx=32, nb=8, nt=160, nshots=2, nh=5, seed=3), 0)


def test_autograd_matches_oracle_gradient_plain_small(ctx):
    # the 100 x 200 problem at its full length: nt = 1500, 11 offsets
    say("case: autograd vs oracle, 100x200 nt1500 nh11")
    _autograd_vs_oracle(ctx, synth.plain_small(), 1)


def test_tape_serves_one_backward(ctx):
    import torch
    import paper_2206_02362_amd as fw
    say("case: tape reuse")
    w = synth.tiny(nz=16, nx=20, nb=4, nt=60, nshots=1, nh=3)
    grid, tv, tg = gpu_problem(w)
    pt = torch.zeros((w.nh, w.nx, w.nz), device="cuda:0")
    data = torch.empty((1, w.nrec, w.nt), device="cuda:0")
    tape = ctx.fwime_forward_tape(grid, tv, tg, w.nh, pt, data)
    a = torch.ones_like(data)
    gv = torch.empty((w.nx, w.nz), device="cuda:0")
    gp = torch.empty_like(pt)
    ctx.fwime_backward_tape(tape, a, gv, gp)
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_backward_tape(tape, a, gv, gp)
    assert e.value.code == fw.FWIME_EINVAL
    tape.free()
    # the forward output equals f(m) + B~ p~ = f(m) for p~ = 0
    ref = ctx.model(grid, tv, tg)
    torch.cuda.synchronize()
    assert torch.equal(data, ref)


def test_autograd_central_differences_full_size(ctx):
    import torch
    import paper_2206_02362_amd as fw
    say("case: autograd FD, 300x1700, 50 shots, nt 5000, 10 directions")
    full = synth.marmousi_set(50, 34)
    w = full
    grid, _, tg = gpu_problem(w)
    m_true = w.vel
    m0 = m_true * (1.0 - 0.02 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 90, 300.0))
    dobs = ctx.model(grid, _dev(m_true), tg)
    pt = _dev(1e-3 * synth.random_ptilde(w.nh, w.nz, w.nx, 91))

    def loss_of(vel_t):
        d = ctx.model(grid, vel_t, tg) + ctx.born_ext_fwd(grid, vel_t, tg, pt)
        return 0.5 * float(((d.double() - dobs.double()) ** 2).sum().item())

    v = _dev(m0).requires_grad_(True)
    d = fw.predicted_data(v, pt, ctx, grid, tg)
    loss = 0.5 * ((d.double() - dobs.double()) ** 2).sum()
    loss.backward()
    grad = v.grad.double().cpu().numpy()
    errs = []
    for seed in range(10):
        xi = synth.gaussian_perturbation(w.nz, w.nx, w.dx, seed, 100.0)
        dm = 1e-3 * m0 * xi
        lp = loss_of(_dev(m0 + dm))
        lm = loss_of(_dev(m0 - dm))
        fd = (lp - lm) / 2.0
        an = float(np.sum(grad * dm))
        errs.append(abs(fd - an) / abs(an))
        say(f"  seed {seed}: fd {fd:.6e} adjoint {an:.6e} rel {errs[-1]:.2e}")
    assert max(errs) < 1e-2
