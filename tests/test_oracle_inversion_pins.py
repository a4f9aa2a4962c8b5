"""Pins of the outer-loop oracle (oracle/inversion.py): the linear spline
operator S, its adjoint S*, and L-BFGS.

Each pin checks the oracle against something other than itself:
* S reproduces every bilinear function a + b z + c x + d z x exactly, on
  non-uniform nodes that are denser around an interface;
* S agrees with scipy's RegularGridInterpolator (linear), a library routine;
* S is the identity when the nodes are the finite-difference grid, and one
  halving of the spacing puts the average of the two neighbours at each
  midpoint (the refinement sequence of Section 2);
* S* is the adjoint of S (dot-product test); refining onto a node set that
  contains the old one leaves the model on the grid unchanged;
* the two-loop recursion equals the explicit BFGS inverse-Hessian update
  applied pair by pair (the textbook dense formula), and satisfies the
  newest secant equation H y = s;
* L-BFGS reaches the known minimizers of a convex quadratic and of the
  Rosenbrock function, with a non-increasing objective, and every accepted
  step meets the strong Wolfe conditions;
* the spline-grid objective's gradient S* grad f(S m) matches central
  differences, on a quadratic and on the FWIME objective.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth
from _helpers import oracle_problem


def _nodes(n, h, coarse, rng, dense_at=None):
    """Node coordinates covering [0, (n-1) h]: spacing `coarse` cells, with
    extra nodes inside the cell span around index `dense_at`."""
    pts = list(np.arange(0, n - 1, coarse) * h) + [(n - 1) * h]
    if dense_at is not None:
        pts += list((dense_at + rng.uniform(-coarse, coarse, 4)) * h)
    pts = np.unique(np.clip(np.round(np.array(pts), 9), 0, (n - 1) * h))
    return pts


@pytest.fixture
def grid():
    rng = np.random.default_rng(3)
    nz, nx, dz, dx = 37, 53, 12.5, 10.0
    zn = _nodes(nz, dz, 8, rng, dense_at=20)
    xn = _nodes(nx, dx, 6, rng)
    return nz, nx, dz, dx, zn, xn


def test_spline_reproduces_bilinear_functions(grid):
    nz, nx, dz, dx, zn, xn = grid
    a, b, c, d = 1500.0, 0.7, -0.3, 1e-3
    fun = lambda x, z: a + b * z + c * x + d * z * x
    mc = fun(xn[:, None], zn[None, :])
    fine = oracle.spline_apply(zn, xn, nz, nx, dz, dx, mc)
    X, Z = np.meshgrid(np.arange(nx) * dx, np.arange(nz) * dz, indexing="ij")
    assert np.max(np.abs(fine - fun(X, Z))) < 1e-9


def test_spline_matches_scipy_linear_interpolator(grid):
    nz, nx, dz, dx, zn, xn = grid
    mc = np.random.default_rng(5).standard_normal((len(xn), len(zn)))
    fine = oracle.spline_apply(zn, xn, nz, nx, dz, dx, mc)
    X, Z = np.meshgrid(np.arange(nx) * dx, np.arange(nz) * dz, indexing="ij")
    ref = RegularGridInterpolator((xn, zn), mc, method="linear")(np.stack([X, Z], -1))
    assert np.max(np.abs(fine - ref)) < 1e-12


def test_spline_identity_on_fd_grid_and_one_halving():
    nz, nx, dz, dx = 17, 21, 10.0, 10.0
    rng = np.random.default_rng(7)
    f = rng.standard_normal((nx, nz))
    zf, xf = np.arange(nz) * dz, np.arange(nx) * dx
    assert np.array_equal(oracle.spline_apply(zf, xf, nz, nx, dz, dx, f), f)
    # nodes every other grid point: node values copied, midpoints averaged
    mc = rng.standard_normal((len(xf[::2]), len(zf[::2])))
    fine = oracle.spline_apply(zf[::2], xf[::2], nz, nx, dz, dx, mc)
    assert np.allclose(fine[::2, ::2], mc, atol=1e-14)
    assert np.allclose(fine[1::2, ::2], 0.5 * (mc[:-1] + mc[1:]), atol=1e-14)
    assert np.allclose(fine[::2, 1::2], 0.5 * (mc[:, :-1] + mc[:, 1:]), atol=1e-14)
    assert np.allclose(fine[1::2, 1::2],
                       0.25 * (mc[:-1, :-1] + mc[1:, :-1] + mc[:-1, 1:] + mc[1:, 1:]), atol=1e-14)


def test_spline_refine_keeps_the_model(grid):
    # a node set containing the coarse one describes the same piecewise-linear
    # model: refining and then mapping to the grid changes nothing
    nz, nx, dz, dx, zn, xn = grid
    rng = np.random.default_rng(11)
    zf = np.unique(np.concatenate([zn, 0.5 * (zn[:-1] + zn[1:])]))
    xf = np.unique(np.concatenate([xn, 0.5 * (xn[:-1] + xn[1:])]))
    mc = rng.standard_normal((len(xn), len(zn)))
    mf = oracle.spline_refine(zn, xn, mc, zf, xf)
    assert np.allclose(mf[::2, ::2], mc, atol=1e-14)
    a = oracle.spline_apply(zn, xn, nz, nx, dz, dx, mc)
    b = oracle.spline_apply(zf, xf, nz, nx, dz, dx, mf)
    assert np.max(np.abs(a - b)) < 1e-12


def test_spline_adjoint_dot_product(grid):
    nz, nx, dz, dx, zn, xn = grid
    rng = np.random.default_rng(9)
    m = rng.standard_normal((len(xn), len(zn)))
    f = rng.standard_normal((nx, nz))
    lhs = float(np.sum(oracle.spline_apply(zn, xn, nz, nx, dz, dx, m) * f))
    rhs = float(np.sum(m * oracle.spline_adjoint(zn, xn, nz, nx, dz, dx, f)))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_spline_rejects_nodes_that_do_not_cover():
    with pytest.raises(ValueError):
        oracle.hat_matrix(np.array([0.0, 50.0]), np.arange(10) * 10.0)
    with pytest.raises(ValueError):
        oracle.hat_matrix(np.array([0.0, 50.0, 40.0, 90.0]), np.arange(10) * 10.0)


def _pairs(n, k, seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((n, n))
    A = q @ q.T + n * np.eye(n)                      # SPD, so every s.y > 0
    S = [rng.standard_normal(n) for _ in range(k)]
    Y = [A @ s for s in S]
    return S, Y, rng.standard_normal(n)


@pytest.mark.parametrize("k", [0, 1, 4])
def test_two_loop_equals_dense_bfgs_update(k):
    n = 9
    S, Y, g = _pairs(n, k, 11 + k)
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1]) if S else 1.0
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):                           # H <- V^T H V + rho s s^T
        rho = 1.0 / float(y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    r = oracle.two_loop(g, S, Y)
    assert np.linalg.norm(r - H @ g) <= 1e-12 * np.linalg.norm(H @ g)
    if S:
        assert np.allclose(oracle.two_loop(Y[-1], S, Y), S[-1], rtol=1e-11, atol=1e-12)


def test_lbfgs_convex_quadratic():
    n = 12
    rng = np.random.default_rng(13)
    q = rng.standard_normal((n, n))
    A = q @ q.T + 0.5 * np.eye(n)
    b = rng.standard_normal(n)
    x, hist = oracle.lbfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(n),
                           memory=5, maxiter=300, gtol=1e-10)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-7 * np.linalg.norm(np.linalg.solve(A, b))
    assert all(b2 <= a2 for a2, b2 in zip(hist, hist[1:]))


def test_lbfgs_rosenbrock():
    def fg(x):
        f = 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
        g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200 * (x[1] - x[0] ** 2)])
        return f, g
    x, hist = oracle.lbfgs(fg, np.array([-1.2, 1.0]), maxiter=200)
    assert np.linalg.norm(x - 1.0) < 1e-6
    assert all(b2 <= a2 for a2, b2 in zip(hist, hist[1:]))


def test_lbfgs_steps_satisfy_strong_wolfe():
    # every accepted step s = x_{k+1} - x_k meets both conditions of the
    # strong Wolfe rule the More-Thuente search is asked for (c1 = 1e-4,
    # c2 = 0.9): sufficient decrease and a small enough directional derivative
    def fg(x):                                       # a smooth non-quadratic convex function
        e = np.exp(0.3 * x)
        return float(np.sum(e - 0.3 * x) + 0.5 * np.sum((x[1:] - x[:-1]) ** 2)), \
            0.3 * e - 0.3 + np.concatenate([[0.0], x[1:] - x[:-1]]) - np.concatenate([x[1:] - x[:-1], [0.0]])
    tr = []
    oracle.lbfgs(fg, np.linspace(-4.0, 6.0, 30), maxiter=40, trace=tr)
    assert len(tr) > 5
    for (x0, f0, g0), (x1, f1, g1) in zip(tr, tr[1:]):
        s = x1 - x0
        assert f1 <= f0 + 1e-4 * float(g0 @ s) + 1e-15 * abs(f0)
        assert abs(float(g1 @ s)) <= 0.9 * abs(float(g0 @ s)) * (1 + 1e-12)


def test_spline_objective_gradient_quadratic(grid):
    nz, nx, dz, dx, zn, xn = grid
    rng = np.random.default_rng(17)
    v0 = rng.standard_normal((nx, nz))
    fg = oracle.on_spline_grid(lambda v: (0.5 * np.sum((v - v0) ** 2), v - v0), zn, xn, nz, nx, dz, dx)
    m = rng.standard_normal(len(xn) * len(zn))
    dm = rng.standard_normal(m.shape)
    f0, g0 = fg(m)
    t = 1e-3
    fd = (fg(m + t * dm)[0] - fg(m - t * dm)[0]) / (2 * t)
    assert abs(fd - g0 @ dm) <= 1e-9 * abs(g0 @ dm)


def test_spline_objective_gradient_fwime():
    # the FWIME objective of a spline-parametrized velocity (eq. fwime.obj
    # evaluated at S m), gradient through S* (eq. fwime.gradient.split)
    w = synth.tiny(nz=16, nx=22, nb=5, nt=110, nshots=2, nh=5, seed=21)
    g, geo = oracle_problem(w)
    true = w.vel + 80.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 22, 30.0)
    dobs = oracle.model(g, true, geo)
    pt = 0.05 * np.random.default_rng(23).standard_normal((w.nh, w.nx, w.nz))
    dso, eps = synth.dso_weights(w.nh), 1e-3
    zn = np.arange(0, w.nz, 5) * w.dz
    zn = np.append(zn, (w.nz - 1) * w.dz) if zn[-1] < (w.nz - 1) * w.dz else zn
    xn = np.arange(0, w.nx, 7) * w.dx
    xn = np.append(xn, (w.nx - 1) * w.dx) if xn[-1] < (w.nx - 1) * w.dx else xn

    def model_fg(v):
        obj, gv, _ = oracle.gradient(g, v, geo, pt, dobs, eps, dso)
        return obj, gv

    fg = oracle.on_spline_grid(model_fg, zn, xn, w.nz, w.nx, w.dz, w.dx)
    m = oracle.spline_adjoint(zn, xn, w.nz, w.nx, w.dz, w.dx, w.vel)
    m /= oracle.spline_adjoint(zn, xn, w.nz, w.nx, w.dz, w.dx, np.ones_like(w.vel))
    m = m.ravel()
    _, gm = fg(m)
    dm = np.random.default_rng(29).standard_normal(m.shape)
    t = 0.1
    fd = (fg(m + t * dm)[0] - fg(m - t * dm)[0]) / (2 * t)
    assert abs(fd - gm @ dm) < 1e-6 * abs(gm @ dm), (fd, gm @ dm)
