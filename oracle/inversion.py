"""FP64 oracle of the FWIME outer loop: the linear spline operator S and its
adjoint, and L-BFGS with a strong-Wolfe line search.

TEST INFRASTRUCTURE ONLY (see the package docstring): never called by the GPU
library, shares no code with it.

Section 2 parametrizes the velocity model on a spline grid: m lives on
coarse nodes and S, a linear spline interpolator, maps it onto the
finite-difference grid (eq. fwime.obj evaluates f(Sm) and B~(Sm)); the
gradient comes back through S* (eq. fwime.gradient.split).  The grids are
refined by halving their spacing, the last one coinciding with the
finite-difference grid, and nodes may be denser near an interface, so the
node coordinates are an input.  Section 3 minimizes with L-BFGS; the step
length comes from a line search for the strong Wolfe conditions (the paper
uses the More-Thuente method).  Readings:

* S is the tensor product of 1D linear (hat-function) interpolations along
  z and x: with node coordinates zn (increasing, covering [0, (nz-1) dz]) and
  xn (covering [0, (nx-1) dx]), fine value (ix, iz) = sum over the four
  surrounding nodes of their bilinear weights.  As matrices, S m = A_x m A_z^T
  with m indexed [x node][z node]; S* f = A_x^T f A_z.
* L-BFGS: the standard two-loop recursion over the last `memory` pairs, the
  initial inverse Hessian scaled by s.y / y.y of the newest pair, pairs with
  s.y <= 0 not kept; the step length from scipy's scalar_search_wolfe1
  (MINPACK's dcsrch, the More-Thuente method) on phi(a) = f(x + a d), with
  c1 = 1e-4, c2 = 0.9, xtol = 1e-14, steps in [0, 1e10] and a first trial
  step of 1.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize._linesearch import scalar_search_wolfe1


def hat_matrix(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """A[i, k]: weight of node k in the linear interpolation at pts[i]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    if np.any(np.diff(nodes) <= 0):
        raise ValueError("nodes must be strictly increasing")
    tol = 1e-9 * max(1.0, abs(nodes[-1] - nodes[0]))
    if pts.min() < nodes[0] - tol or pts.max() > nodes[-1] + tol:
        raise ValueError("nodes must cover every grid point")
    A = np.zeros((len(pts), len(nodes)))
    for i, p in enumerate(pts):
        if len(nodes) == 1:
            A[i, 0] = 1.0
            continue
        k = int(np.clip(np.searchsorted(nodes, p, side="right") - 1, 0, len(nodes) - 2))
        t = (p - nodes[k]) / (nodes[k + 1] - nodes[k])
        t = min(max(t, 0.0), 1.0)
        A[i, k] += 1.0 - t
        A[i, k + 1] += t
    return A


def spline_matrices(zn, xn, nz: int, nx: int, dz: float, dx: float):
    return hat_matrix(zn, np.arange(nz) * dz), hat_matrix(xn, np.arange(nx) * dx)


def spline_apply(zn, xn, nz: int, nx: int, dz: float, dx: float, mc: np.ndarray) -> np.ndarray:
    """S m: node values mc [len(xn)][len(zn)] onto the model grid [nx][nz]."""
    Az, Ax = spline_matrices(zn, xn, nz, nx, dz, dx)
    return Ax @ np.asarray(mc, dtype=np.float64) @ Az.T


def spline_adjoint(zn, xn, nz: int, nx: int, dz: float, dx: float, f: np.ndarray) -> np.ndarray:
    """S* f: a model-grid field [nx][nz] onto the nodes [len(xn)][len(zn)]."""
    Az, Ax = spline_matrices(zn, xn, nz, nx, dz, dx)
    return Ax.T @ np.asarray(f, dtype=np.float64) @ Az


def spline_refine(zn, xn, mc: np.ndarray, zn_fine, xn_fine) -> np.ndarray:
    """Node values mc [len(xn)][len(zn)] onto a finer node set [len(xn_fine)][len(zn_fine)]:
    the same linear interpolation evaluated at the new nodes (the next grid of
    the coarse-to-fine sequence)."""
    Az = hat_matrix(zn, zn_fine)
    Ax = hat_matrix(xn, xn_fine)
    return Ax @ np.asarray(mc, dtype=np.float64) @ Az.T


def two_loop(g: np.ndarray, S, Y) -> np.ndarray:
    """H g for the L-BFGS inverse-Hessian approximation H built from the pairs
    (s_i, y_i), oldest first, with H_0 = (s.y / y.y of the newest pair) I, or I
    without pairs; the two-loop recursion, which never forms H."""
    q = np.asarray(g, dtype=np.float64).copy()
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        rho = 1.0 / float(y @ s)
        a = rho * float(s @ q)
        alphas.append((a, rho, s, y))
        q -= a * y
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1]) if S else 1.0
    r = gamma * q
    for a, rho, s, y in reversed(alphas):
        b = rho * float(y @ r)
        r += (a - b) * s
    return r


def lbfgs(fun_grad, x0: np.ndarray, memory: int = 5, maxiter: int = 100, gtol: float = 1e-8, trace=None):
    """Minimize fun_grad(x) -> (f, g) by L-BFGS; returns (x, [f per iterate]).
    A list passed as `trace` receives (x, f, g) of every iterate.

    Stops when ||g|| <= gtol ||g_0||, after maxiter iterations, or when the line
    search finds no step (the paper then refines the spline grid)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    cache = {}

    def fg(z):
        key = z.tobytes()
        if key not in cache:
            cache.clear()
            f, g = fun_grad(z)
            cache[key] = (float(f), np.asarray(g, dtype=np.float64))
        return cache[key]

    f, g = fg(x)
    g0 = np.linalg.norm(g)
    hist = [f]
    if trace is not None:
        trace.append((x.copy(), f, g.copy()))
    S, Y = [], []
    for _ in range(maxiter):
        if np.linalg.norm(g) <= gtol * g0:
            break
        d = -two_loop(g, S, Y)
        step = scalar_search_wolfe1(lambda a: fg(x + a * d)[0], lambda a: float(fg(x + a * d)[1] @ d),
                                    phi0=f, derphi0=float(g @ d), c1=1e-4, c2=0.9,
                                    amax=1e10, amin=0.0, xtol=1e-14)[0]
        if step is None:
            break
        x_new = x + step * d
        f_new, g_new = fg(x_new)
        s_k, y_k = x_new - x, g_new - g
        if float(s_k @ y_k) > 1e-12 * float(np.linalg.norm(s_k) * np.linalg.norm(y_k)):
            S.append(s_k)
            Y.append(y_k)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = x_new, f_new, g_new
        hist.append(f)
        if trace is not None:
            trace.append((x.copy(), f, g.copy()))
    return x, hist


def on_spline_grid(fun_grad_model, zn, xn, nz: int, nx: int, dz: float, dx: float):
    """The objective of a model-grid function seen from the spline nodes:
    m -> (f(S m), S* grad f(S m)), node values flattened [len(xn) * len(zn)]."""
    Az, Ax = spline_matrices(zn, xn, nz, nx, dz, dx)
    shape = (len(xn), len(zn))

    def fg(mc):
        f, g = fun_grad_model(Ax @ np.reshape(mc, shape) @ Az.T)
        return f, (Ax.T @ np.asarray(g, dtype=np.float64) @ Az).ravel()

    return fg
