"""L-BFGS search direction on the GPU (fwime_lbfgs_direction) against the
FP64 oracle's two-loop recursion, and the L-BFGS driver
(fwime_lbfgs_minimize) against the oracle's L-BFGS with the More-Thuente
search: on a quadratic, and as the method's outer loop on the FWIME objective
of a spline-parametrized velocity.

Pairs come from a symmetric positive-definite operator (y = A s), so every
curvature s.y is positive.  Tolerance: relative L2 <= 1e-5 (FP32 vectors,
FP64 inner products); lengths span many 256-thread blocks with a ragged tail.
"""
import sys

import numpy as np
import pytest

import oracle
from _helpers import rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_02362_amd as fw
    c = fw.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def _pairs(n, k, seed):
    # A = diag(a) + u u^T with a in [0.5, 20]: SPD, applied without forming it
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 20.0, n)
    u = rng.standard_normal(n) / np.sqrt(n)
    S = rng.standard_normal((k, n)).astype(np.float32)
    Y = np.array([a * s + u * (u @ s) for s in S.astype(np.float64)]).reshape(k, n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    return S, Y, g


@pytest.mark.parametrize("n,k", [(6131, 0), (6131, 1), (6131, 5), (1_000_003, 5), (70_001, 20)])
def test_lbfgs_direction_matches_oracle(ctx, n, k):
    say(f"case: lbfgs direction n {n}, {k} pairs")
    S, Y, g = _pairs(n, k, n + k)
    ref = -oracle.two_loop(g.astype(np.float64), [s.astype(np.float64) for s in S],
                           [y.astype(np.float64) for y in Y])
    out = ctx.lbfgs_direction(dev(S) if k else None, dev(Y) if k else None, dev(g))
    err = rel_l2(out.double().cpu().numpy(), ref)
    say(f"  rel-L2 {err:.3e}")
    assert err < TOL


def test_lbfgs_direction_in_place_and_descent(ctx):
    S, Y, g = _pairs(20_000, 4, 3)
    gd = dev(g)
    d = ctx.lbfgs_direction(dev(S), dev(Y), gd)
    ctx.fwime_lbfgs_direction(dev(S), dev(Y), gd, gd)          # d_out = g
    import torch
    assert torch.equal(d, gd)
    assert float((d.double() * dev(g).double()).sum()) < 0     # H is positive definite


def test_lbfgs_direction_rejects_nonpositive_curvature(ctx):
    import paper_2206_02362_amd as fw
    S, Y, g = _pairs(5000, 3, 9)
    Y[1] = -Y[1]
    out = dev(np.full(5000, 3.0))
    with pytest.raises(fw.FwimeError):
        ctx.fwime_lbfgs_direction(dev(S), dev(Y), dev(g), out)
    assert float(out.min()) == 3.0 and float(out.max()) == 3.0


def test_lbfgs_minimize_quadratic_matches_oracle(ctx):
    # f = x.A x / 2 - b.x with A = diag(a) + u u^T: the oracle's L-BFGS (FP64,
    # MINPACK's More-Thuente search) and the library's take the same first
    # iterates, and both reach A^-1 b (Sherman-Morrison)
    import torch
    n = 50_000
    rng = np.random.default_rng(21)
    a = rng.uniform(1.0, 10.0, n)
    u = rng.standard_normal(n) / np.sqrt(n)
    b = rng.standard_normal(n)
    x0 = 0.1 * rng.standard_normal(n)
    a, u, b, x0 = (v.astype(np.float32).astype(np.float64) for v in (a, u, b, x0))
    say(f"case: lbfgs minimize quadratic n {n}")
    at, ut, bt = dev(a), dev(u), dev(b)

    def fg_dev(x):
        ax = at * x + ut * torch.dot(ut, x)
        return float(0.5 * torch.dot(x.double(), ax.double()) - torch.dot(bt.double(), x.double())), ax - bt

    def fg_ref(x):
        ax = a * x + u * (u @ x)
        return 0.5 * x @ ax - b @ x, ax - b

    x, hist, iters = ctx.lbfgs_minimize(fg_dev, dev(x0), memory=5, maxiter=30, gtol=1e-5)
    _, ref = oracle.lbfgs(fg_ref, x0, memory=5, maxiter=30, gtol=1e-5)
    sol = b / a - (u / a) * ((u @ (b / a)) / (1.0 + u @ (u / a)))
    err = rel_l2(x.double().cpu().numpy(), sol)
    say(f"  {iters} iterations (oracle {len(ref) - 1}), rel-L2 to the solution {err:.3e}, "
        f"f {hist[:4]} vs {ref[:4]}")
    assert np.allclose(hist[:4], ref[:4], rtol=1e-5)
    assert all(q <= p for p, q in zip(hist, hist[1:]))
    assert err < 1e-4


def test_lbfgs_minimize_fwime_on_spline_grid(ctx):
    # the outer loop of the method: FWIME objective of the spline-parametrized
    # velocity, gradient through S* (spline apply, gradient, spline adjoint,
    # all through the library), two iterations from the background model
    import torch
    import synth
    from _helpers import gpu_problem, oracle_problem_f32
    say("case: lbfgs minimize FWIME on a spline grid, 16x22 nt110 2 shots")
    w = synth.tiny(nz=16, nx=22, nb=5, nt=110, nshots=2, nh=5, seed=21)
    g, geo, vel = oracle_problem_f32(w)
    grid, tv, tg = gpu_problem(w)
    true = w.vel + 80.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 22, 30.0)
    dobs = ctx.model(grid, dev(true), tg)
    pt = dev(0.05 * np.random.default_rng(23).standard_normal((w.nh, w.nx, w.nz)))
    dso, eps = synth.dso_weights(w.nh), 1e-3
    zn = np.append(np.arange(0, w.nz - 1, 5) * w.dz, (w.nz - 1) * w.dz)
    xn = np.append(np.arange(0, w.nx - 1, 7) * w.dx, (w.nx - 1) * w.dx)

    def fg(m):
        v = ctx.spline_apply(w.nz, w.nx, w.dz, w.dx, zn, xn, m)
        obj, gv, _ = ctx.gradient(grid, v, tg, pt, dobs, eps, dso)
        return float(obj), ctx.spline_adjoint(w.nz, w.nx, w.dz, w.dx, zn, xn, gv.contiguous())

    m0 = torch.full((len(xn), len(zn)), float(np.mean(w.vel)), device="cuda:0")
    f0 = oracle.objective(g, oracle.spline_apply(zn, xn, w.nz, w.nx, w.dz, w.dx, m0.double().cpu().numpy()),
                          geo, pt.double().cpu().numpy(), dobs.double().cpu().numpy(), eps, dso)
    m, hist, iters = ctx.lbfgs_minimize(fg, m0, memory=3, maxiter=2)
    # the oracle's outer loop on the same problem (FP64 throughout)
    dobs64, pt64 = dobs.double().cpu().numpy(), pt.double().cpu().numpy()

    def model_fg(v):
        obj, gv, _ = oracle.gradient(g, v, geo, pt64, dobs64, eps, dso)
        return obj, gv

    _, ref = oracle.lbfgs(oracle.on_spline_grid(model_fg, zn, xn, w.nz, w.nx, w.dz, w.dx),
                          m0.double().cpu().numpy().ravel(), memory=3, maxiter=2)
    say(f"  {iters} iterations, objective {hist}, oracle {ref}")
    assert abs(hist[0] - f0) <= 1e-4 * abs(f0)
    assert iters >= 1 and hist[-1] < hist[0]
    assert len(hist) == len(ref) and np.allclose(hist, ref, rtol=1e-4)
    assert all(q <= p for p, q in zip(hist, hist[1:]))


def test_lbfgs_minimize_rejects_small_workspace(ctx):
    import ctypes
    import torch
    import paper_2206_02362_amd as fw
    from paper_2206_02362_amd import _abi
    n, memory = 1000, 4
    x = dev(np.ones(n))
    work = torch.empty(_abi.LBFGS_WORK_HEAD + (2 * memory + 6) * n - 1, device="cuda:0")
    hist = np.zeros(3)
    iters = ctypes.c_int32(-1)
    cb = _abi.OBJECTIVE_FN(lambda user, xp, gp, fp: 1)       # never reached
    rc = ctx._lib.fwime_lbfgs_minimize(ctx._h, n, memory, 2, 0.0, cb, None, x.data_ptr(), work.data_ptr(),
                                       work.numel(), hist.ctypes.data, ctypes.byref(iters),
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == fw.FWIME_EINVAL and iters.value == -1
    assert "work needs" in ctx._lib.fwime_last_error(ctx._h).decode()
