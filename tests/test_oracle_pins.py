"""Pins of the FP64 oracle against what mathematics and the paper fix.

None of these compare the oracle with itself: each checks an independent
property (a textbook formula, an analytic solution, an adjoint identity, a
derivative, a symmetry) chosen so that a dropped term, a wrong sign, a wrong
index or a transposed operand in the oracle fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from _helpers import dot_err, oracle_problem, rel_l2


# ---------------------------------------------------------------------------
# Stencil
# ---------------------------------------------------------------------------

def test_fornberg_weights_textbook():
    # Central second-derivative weights tabulated by Fornberg (1988), Table 1.
    assert oracle.fd_second_derivative_weights(1) == [Fraction(-2), Fraction(1)]
    assert oracle.fd_second_derivative_weights(2) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]
    assert oracle.fd_second_derivative_weights(4) == [
        Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)]


def test_laplacian_eighth_order():
    # Error of the discrete Laplacian of sin(a x) sin(b z) on an interior patch
    # must fall by 2^8 when the spacing halves.
    errs = []
    for d in (0.3, 0.15):
        n = int(round(12.0 / d))
        x = np.arange(n) * d
        X, Z = np.meshgrid(x, x, indexing="ij")
        a, b = 1.3, 0.7
        u = np.sin(a * X) * np.sin(b * Z)
        lap = oracle.laplacian(u, d, d)
        exact = -(a * a + b * b) * u
        sl = (slice(10, n - 10), slice(10, n - 10))
        errs.append(np.max(np.abs(lap[sl] - exact[sl])))
    order = math.log2(errs[0] / errs[1])
    assert abs(order - 8.0) < 0.3, order


def test_laplacian_zero_outside():
    # A single 1 in the corner: the Laplacian sees zeros outside the array.
    u = np.zeros((12, 12))
    u[0, 0] = 1.0
    lap = oracle.laplacian(u, 2.0, 3.0)
    w = [float(x) for x in oracle.fd_second_derivative_weights(4)]
    assert lap[0, 0] == pytest.approx(w[0] * (1 / 4 + 1 / 9))
    assert lap[0, 3] == pytest.approx(w[3] / 4)
    assert lap[2, 0] == pytest.approx(w[2] / 9)
    assert lap[5, 0] == 0.0


def test_cfl_limit_value_and_stability():
    # Closed form for dx = dz: v dt / dx <= 2 / sqrt(2 * 6.50158...) = 0.5546...
    nyq = 205 / 72 + 2 * (8 / 5 + 1 / 5 + 8 / 315 + 1 / 560)
    assert oracle.cfl_limit(10.0, 10.0) == pytest.approx(10.0 * 2 / math.sqrt(2 * nyq), rel=1e-14)
    assert oracle.cfl_limit(10.0, 10.0) / 10.0 == pytest.approx(0.5546, abs=1e-4)

    # Growth test on a periodic-free random field: just below the limit stays
    # bounded, clearly above it blows up.
    def run(courant):
        rng = np.random.default_rng(0)
        n = 48
        u_prev = np.zeros((n, n))
        u = rng.standard_normal((n, n))
        V = (courant * 10.0) ** 2
        for _ in range(400):
            u_prev, u = u, 2 * u - u_prev + V * oracle.laplacian(u, 10.0, 10.0)
        return np.max(np.abs(u))
    lim = oracle.cfl_limit(10.0, 10.0) / 10.0
    assert run(0.98 * lim) < 1e3
    assert run(1.05 * lim) > 1e6


def test_sponge_profile():
    g = oracle.sponge_profile(10, 20, 0.3)
    assert g.shape == (50,)
    assert np.all(g[20:30] == 1.0)
    assert g[0] == pytest.approx(math.exp(-0.09))
    assert g[49] == pytest.approx(math.exp(-0.09))
    assert g[19] == pytest.approx(math.exp(-(0.3 / 20) ** 2))
    assert np.all(np.diff(g[:21]) > 0)


def test_pad_edge_adjoint_dot():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((7, 5))
    b = rng.standard_normal((7 + 6, 5 + 6))
    lhs = np.sum(oracle.pad_edge(a, 3) * b)
    rhs = np.sum(a * oracle.pad_edge_adjoint(b, 3))
    assert dot_err(lhs, rhs) < 1e-13
    assert oracle.pad_edge(a, 3)[0, 0] == a[0, 0]
    assert oracle.pad_edge(a, 3)[-1, 4] == a[-1, 1]


# ---------------------------------------------------------------------------
# Propagator
# ---------------------------------------------------------------------------

def analytic_green_2d(r, c, t, f_peak, n_quad=600):
    """u(r,t) for (1/c^2) u_tt - Laplacian u = delta(x) w(t), w = Ricker:
    u = 1/(2 pi) int_0^{acosh(ct/r)} w(t - (r/c) cosh th) dth  (t > r/c)."""
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    out = np.zeros_like(t)
    for i, ti in enumerate(t):
        if c * ti <= r:
            continue
        thmax = math.acosh(c * ti / r)
        th = 0.5 * thmax * (xg + 1.0)
        vals = synth.ricker_value(ti - (r / c) * np.cosh(th), f_peak)
        out[i] = 0.5 * thmax * np.sum(wg * vals) / (2 * math.pi)
    return out


def _homogeneous(nz, nx, nb, nt, dx, dt, c, src, recs, f_peak, alpha=0.3):
    g = oracle.Grid(nz, nx, nb, nt, dx, dx, dt, alpha)
    vel = np.full((nx, nz), c)
    rec = np.asarray(recs, dtype=np.int32)
    geo = oracle.Geometry(np.array([src[0]], np.int32), np.array([src[1]], np.int32),
                          rec[None, :, 0], rec[None, :, 1],
                          synth.ricker(nt, dt, f_peak)[None])
    return g, vel, geo


def test_green_function_homogeneous():
    # 10 Hz Ricker, 2000 m/s, 10 m grid (8 points per shortest wavelength at
    # 25 Hz), receivers 400 m from the source along x and along the diagonal;
    # the window ends before waves from the padded edges come back.
    c, dx, dt, nt, f = 2000.0, 10.0, 1e-3, 600, 10.0
    nz = nx = 201
    src = (100, 100)
    recs = [(100, 140), (72, 128)]
    g, vel, geo = _homogeneous(nz, nx, 20, nt, dx, dt, c, src, recs, f)
    d = oracle.model(g, vel, geo)[0]
    t = np.arange(nt) * dt
    for k, (iz, ix) in enumerate(recs):
        r = dx * math.hypot(iz - src[0], ix - src[1])
        ref = analytic_green_2d(r, c, t, f)
        assert rel_l2(d[k], ref) < 1e-2


def test_green_function_grid_convergence():
    # Fixed Courant number 0.2: halving dx halves dt; the 8th-order space error
    # is negligible, so the error against the analytic solution must fall as
    # dt^2 (order 2).
    c, f, L, r = 2000.0, 6.0, 1600.0, 300.0
    T = 0.55
    errs = []
    for dx in (20.0, 10.0, 5.0):
        dt = 0.2 * dx / c
        n = int(round(L / dx)) + 1
        mid = n // 2
        off = int(round(r / dx))
        nt = int(round(T / dt)) + 1
        g, vel, geo = _homogeneous(n, n, int(round(200 / dx)), nt, dx, dt, c, (mid, mid), [(mid, mid + off)], f)
        d = oracle.model(g, vel, geo)[0, 0]
        t = np.arange(nt) * dt
        keep = slice(None, None, int(round(0.01 / dt)))
        ref = analytic_green_2d(r, c, t[keep], f)
        errs.append(np.linalg.norm(d[keep] - ref) / np.linalg.norm(ref))
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert abs(o1 - 2.0) < 0.3 and abs(o2 - 2.0) < 0.3, (errs, o1, o2)


def test_reciprocity_heterogeneous_with_sponge():
    w = synth.tiny(nz=30, nx=40, nb=10, nt=250, nshots=1)
    g, _ = oracle_problem(w)
    A, B = (3, 6), (21, 33)
    wav = synth.ricker(w.nt, w.dt, 25.0)[None]

    def shot(s, r):
        geo = oracle.Geometry(np.array([s[0]]), np.array([s[1]]), np.array([[r[0]]]), np.array([[r[1]]]), wav)
        return oracle.model(g, w.vel, geo)[0, 0]
    ab, ba = shot(A, B), shot(B, A)
    assert np.max(np.abs(ab)) > 0
    assert rel_l2(ab, ba) < 1e-12


# ---------------------------------------------------------------------------
# Adjoint (dot-product) tests
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    w = synth.tiny(nz=20, nx=28, nb=6, nt=120, nshots=2, nh=5)
    g, geo = oracle_problem(w)
    return w, g, geo


def test_dot_wavelet_modeling(small):
    w, g, geo = small
    rng = np.random.default_rng(11)
    wav = rng.standard_normal(w.wavelet.shape)
    geo2 = oracle.Geometry(geo.src_iz, geo.src_ix, geo.rec_iz, geo.rec_ix, wav)
    d = rng.standard_normal((w.nshots, w.nrec, w.nt))
    lhs = np.sum(oracle.model(g, w.vel, geo2) * d)
    rhs = np.sum(wav * oracle.model_adjoint_wavelet(g, w.vel, geo2, d))
    assert dot_err(lhs, rhs) < 1e-10


def test_dot_born(small):
    w, g, geo = small
    rng = np.random.default_rng(12)
    dv = rng.standard_normal((w.nx + 2 * w.nb, w.nz + 2 * w.nb))
    d = rng.standard_normal((w.nshots, w.nrec, w.nt))
    lhs = np.sum(oracle.born(g, w.vel, geo, dv) * d)
    rhs = np.sum(dv * oracle.born_adjoint(g, w.vel, geo, d))
    assert dot_err(lhs, rhs) < 1e-10


def test_dot_born_extended(small):
    w, g, geo = small
    rng = np.random.default_rng(13)
    pt = rng.standard_normal((w.nh, w.nx, w.nz))
    d = rng.standard_normal((w.nshots, w.nrec, w.nt))
    lhs = np.sum(oracle.born_ext_fwd(g, w.vel, geo, pt) * d)
    rhs = np.sum(pt * oracle.born_ext_adj(g, w.vel, geo, d, w.nh))
    assert dot_err(lhs, rhs) < 1e-10


def test_dot_born_extended_offsets_leave_grid():
    # nb smaller than H: some y -/+ h fall outside the padded grid and are dropped.
    w = synth.tiny(nz=12, nx=14, nb=3, nt=90, nshots=1, nh=11)
    g, geo = oracle_problem(w)
    rng = np.random.default_rng(14)
    pt = rng.standard_normal((w.nh, w.nx, w.nz))
    d = rng.standard_normal((1, w.nrec, w.nt))
    lhs = np.sum(oracle.born_ext_fwd(g, w.vel, geo, pt) * d)
    rhs = np.sum(pt * oracle.born_ext_adj(g, w.vel, geo, d, w.nh))
    assert dot_err(lhs, rhs) < 1e-10


# ---------------------------------------------------------------------------
# Linearizations
# ---------------------------------------------------------------------------

def test_born_is_derivative_of_modeling(small):
    # || f(m + t dm) - f(m) - t B P dm || must shrink as t^2.
    w, g, geo = small
    dm = 50.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 5, 40.0)
    f0 = oracle.model(g, w.vel, geo)
    bd = oracle.born(g, w.vel, geo, oracle.pad_edge(dm, w.nb))
    res = []
    for t in (0.4, 0.2, 0.1):
        ft = oracle.model(g, w.vel + t * dm, geo)
        res.append(np.linalg.norm(ft - f0 - t * bd))
    s1 = math.log2(res[0] / res[1])
    s2 = math.log2(res[1] / res[2])
    assert abs(s1 - 2) < 0.1 and abs(s2 - 2) < 0.1, (res, s1, s2)


def test_extended_born_zero_offset_is_born(small):
    w, g, geo = small
    rng = np.random.default_rng(15)
    dv = rng.standard_normal((w.nx, w.nz))
    pt = np.zeros((w.nh, w.nx, w.nz))
    pt[w.nh // 2] = dv
    dv_pad = np.zeros((w.nx + 2 * w.nb, w.nz + 2 * w.nb))
    dv_pad[w.nb:w.nb + w.nx, w.nb:w.nb + w.nz] = dv
    assert rel_l2(oracle.born_ext_fwd(g, w.vel, geo, pt), oracle.born(g, w.vel, geo, dv_pad)) < 1e-12


def test_extended_born_linear(small):
    w, g, geo = small
    rng = np.random.default_rng(16)
    a = rng.standard_normal((w.nh, w.nx, w.nz))
    b = rng.standard_normal((w.nh, w.nx, w.nz))
    lhs = oracle.born_ext_fwd(g, w.vel, geo, 2.0 * a - 3.0 * b)
    rhs = 2.0 * oracle.born_ext_fwd(g, w.vel, geo, a) - 3.0 * oracle.born_ext_fwd(g, w.vel, geo, b)
    assert rel_l2(lhs, rhs) < 1e-12


def test_extended_born_offset_is_a_source_shift():
    # In a homogeneous medium with no taper, a single extended spike at
    # (z1, y0, h0) scatters the incident field found at y0 - h0 into y0 + h0.
    # Translating the source by 2 h0 moves that incident field onto y0 + h0,
    # so the extended response equals the ordinary Born response of a spike at
    # (z1, y0 + h0) for the shifted source.  Exact while the numerical domain of
    # dependence (4 cells per step) stays inside the grid.
    c, dx, dt, nt = 2500.0, 10.0, 2e-3, 40
    n = 2 * 4 * nt + 40
    g = oracle.Grid(n, n, 1, nt, dx, dx, dt, 0.0)
    vel = np.full((n, n), c)
    mid = n // 2
    h0 = 3
    z1, y0 = mid, mid
    wav = synth.ricker(nt, dt, 40.0)[None]
    recs = np.array([[mid - 4, mid - 2, mid + 3]], np.int32)
    rec_iz = np.full((1, 3), mid - 4, np.int32)
    xs = mid - h0 - 4
    nh = 2 * h0 + 1
    pt = np.zeros((nh, n, n))
    pt[2 * h0, y0, z1] = 7.0           # ih = +h0
    geo = oracle.Geometry(np.array([mid - 4]), np.array([xs]), rec_iz, recs, wav)
    d_ext = oracle.born_ext_fwd(g, vel, geo, pt)
    dv = np.zeros((n + 2, n + 2))
    dv[1 + y0 + h0, 1 + z1] = 7.0
    geo_shift = oracle.Geometry(np.array([mid - 4]), np.array([xs + 2 * h0]), rec_iz, recs, wav)
    d_born = oracle.born(g, vel, geo_shift, dv)
    assert np.max(np.abs(d_born)) > 0
    assert rel_l2(d_ext, d_born) < 1e-10


def test_extended_born_mirror_symmetry(small):
    # Flipping x for model and geometry maps p~(y, h) to p~(nx-1-y, -h).
    w, g, geo = small
    rng = np.random.default_rng(17)
    pt = rng.standard_normal((w.nh, w.nx, w.nz))
    d = oracle.born_ext_fwd(g, w.vel, geo, pt)
    geo_f = oracle.Geometry(geo.src_iz, w.nx - 1 - geo.src_ix, geo.rec_iz, w.nx - 1 - geo.rec_ix, geo.wavelet)
    d_f = oracle.born_ext_fwd(g, w.vel[::-1].copy(), geo_f, pt[::-1, ::-1].copy())
    assert rel_l2(d_f, d) < 1e-12


# ---------------------------------------------------------------------------
# FWIME objective and gradient
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def grad_case():
    w = synth.tiny(nz=16, nx=22, nb=5, nt=110, nshots=2, nh=5, seed=21)
    g, geo = oracle_problem(w)
    true = w.vel + 80.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 22, 30.0)
    dobs = oracle.model(g, true, geo)
    rng = np.random.default_rng(23)
    pt = 0.05 * rng.standard_normal((w.nh, w.nx, w.nz))
    dso = synth.dso_weights(w.nh)
    eps = 1e-3
    out = oracle.gradient(g, w.vel, geo, pt, dobs, eps, dso)
    return w, g, geo, dobs, pt, dso, eps, out


def test_gradient_objective_value(grad_case):
    w, g, geo, dobs, pt, dso, eps, (obj, gv, gp) = grad_case
    assert obj == pytest.approx(oracle.objective(g, w.vel, geo, pt, dobs, eps, dso), rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_velocity_central_difference(grad_case, seed):
    w, g, geo, dobs, pt, dso, eps, (obj, gv, gp) = grad_case
    # central-difference error falls as t^2 (about 5e-8 at t = 0.1 m/s)
    dm = synth.gaussian_perturbation(w.nz, w.nx, w.dx, 100 + seed, 30.0)
    t = 0.1
    fp = oracle.objective(g, w.vel + t * dm, geo, pt, dobs, eps, dso)
    fm = oracle.objective(g, w.vel - t * dm, geo, pt, dobs, eps, dso)
    fd = (fp - fm) / (2 * t)
    an = float(np.sum(gv * dm))
    assert abs(fd - an) / abs(an) < 1e-6, (fd, an)


def test_gradient_ptilde_central_difference(grad_case):
    w, g, geo, dobs, pt, dso, eps, (obj, gv, gp) = grad_case
    rng = np.random.default_rng(31)
    dp = rng.standard_normal(pt.shape)
    t = 0.1
    fp = oracle.objective(g, w.vel, geo, pt + t * dp, dobs, eps, dso)
    fm = oracle.objective(g, w.vel, geo, pt - t * dp, dobs, eps, dso)
    fd = (fp - fm) / (2 * t)
    an = float(np.sum(gp * dp))
    assert abs(fd - an) / abs(an) < 1e-9, (fd, an)


def test_gradient_ptilde_zero_is_fwi(grad_case):
    # With p~ = 0 the objective is the FWI misfit and the velocity gradient is
    # P^T B^T (f(m) - d_obs) (the eps -> infinity limit of the method).
    w, g, geo, dobs, pt, dso, eps, _ = grad_case
    zero = np.zeros_like(pt)
    obj, gv, gp = oracle.gradient(g, w.vel, geo, zero, dobs, 0.7, dso)
    r = oracle.model(g, w.vel, geo) - dobs
    assert obj == pytest.approx(0.5 * np.sum(r * r), rel=1e-13)
    ref = oracle.pad_edge_adjoint(oracle.born_adjoint(g, w.vel, geo, r), w.nb)
    assert rel_l2(gv, ref) < 1e-12
    assert rel_l2(gp, oracle.born_ext_adj(g, w.vel, geo, r, w.nh)) < 1e-12


# the gradient with time lags: central differences in m (error ~ t^2) and in
# p~, and a single lag against the single offset (the same scattering source)
@pytest.fixture(scope="module")
def grad_case_tau():
    w = synth.tiny(nz=16, nx=22, nb=5, nt=110, nshots=2, nh=5, seed=21)
    g, geo = oracle_problem(w)
    true = w.vel + 80.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 22, 30.0)
    dobs = oracle.model(g, true, geo)
    rng = np.random.default_rng(24)
    pt = 0.05 * rng.standard_normal((5, w.nx, w.nz))
    dso = synth.dso_weights(5)
    eps, lag = 1e-3, 6
    out = oracle.gradient(g, w.vel, geo, pt, dobs, eps, dso, lag=lag)
    return w, g, geo, dobs, pt, dso, eps, lag, out


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_time_lag_velocity_central_difference(grad_case_tau, seed):
    w, g, geo, dobs, pt, dso, eps, lag, (obj, gv, gp) = grad_case_tau
    assert obj == pytest.approx(oracle.objective(g, w.vel, geo, pt, dobs, eps, dso, lag=lag), rel=1e-13)
    dm = synth.gaussian_perturbation(w.nz, w.nx, w.dx, 200 + seed, 30.0)
    t = 0.1
    fp = oracle.objective(g, w.vel + t * dm, geo, pt, dobs, eps, dso, lag=lag)
    fm = oracle.objective(g, w.vel - t * dm, geo, pt, dobs, eps, dso, lag=lag)
    fd = (fp - fm) / (2 * t)
    an = float(np.sum(gv * dm))
    assert abs(fd - an) / abs(an) < 1e-6, (fd, an)


def test_gradient_time_lag_ptilde_central_difference(grad_case_tau):
    w, g, geo, dobs, pt, dso, eps, lag, (obj, gv, gp) = grad_case_tau
    dp = np.random.default_rng(32).standard_normal(pt.shape)
    t = 0.1
    fp = oracle.objective(g, w.vel, geo, pt + t * dp, dobs, eps, dso, lag=lag)
    fm = oracle.objective(g, w.vel, geo, pt - t * dp, dobs, eps, dso, lag=lag)
    fd = (fp - fm) / (2 * t)
    an = float(np.sum(gp * dp))
    assert abs(fd - an) / abs(an) < 1e-9, (fd, an)


def test_gradient_single_lag_equals_single_offset(grad_case_tau):
    w, g, geo, dobs, pt, dso, eps, lag, _ = grad_case_tau
    one = pt[2:3]
    a = oracle.gradient(g, w.vel, geo, one, dobs, eps, dso[2:3], lag=lag)
    b = oracle.gradient(g, w.vel, geo, one, dobs, eps, dso[2:3])
    assert a[0] == pytest.approx(b[0], rel=1e-13)
    assert rel_l2(a[1], b[1]) < 1e-12 and rel_l2(a[2], b[2]) < 1e-12


# ---------------------------------------------------------------------------
# Variable-projection step (eqs. vp.obj, pert.opt): linear CG on the normal
# equation, pinned against the normal matrix assembled column by column and a
# direct solve
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module", params=[None, 4], ids=["offsets", "time-lags"])
def vp_case(request):
    # the normal matrix assembled column by column, for the offset extension
    # and for time lags (3 lags of 4 steps)
    lag = request.param
    w = synth.tiny(nz=4, nx=6, nb=3, nt=50, nshots=2, nh=3, seed=21)
    g, geo = oracle_problem(w)
    true = w.vel * (1.0 + 0.05 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 22, 20.0))
    dobs = oracle.model(g, true, geo)
    if lag is None:
        fwd = lambda x: oracle.born_ext_fwd(g, w.vel, geo, x)
        adj = lambda d: oracle.born_ext_adj(g, w.vel, geo, d, w.nh)
    else:
        fwd = lambda x: oracle.born_ext_tau_fwd(g, w.vel, geo, x, lag)
        adj = lambda d: oracle.born_ext_tau_adj(g, w.vel, geo, d, w.nh, lag)
    n = w.nh * w.nx * w.nz
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(adj(fwd(e.reshape(w.nh, w.nx, w.nz))).ravel())
    H0 = np.array(cols).T                          # B~* B~, column i = B~* B~ e_i
    b = adj(dobs - oracle.model(g, w.vel, geo)).ravel()
    return w, g, geo, dobs, H0, b, lag


def test_vp_normal_operator_symmetric_psd(vp_case):
    w, g, geo, dobs, H0, b, lag = vp_case
    assert np.linalg.norm(H0 - H0.T) <= 1e-10 * np.linalg.norm(H0)
    ev = np.linalg.eigvalsh(0.5 * (H0 + H0.T))
    assert ev.min() >= -1e-10 * ev.max() and ev.max() > 0


def test_vp_cg_reaches_direct_solution(vp_case):
    w, g, geo, dobs, H0, b, lag = vp_case
    dso = synth.dso_weights(w.nh)
    lam = np.linalg.eigvalsh(0.5 * (H0 + H0.T)).max()
    eps = math.sqrt(0.1 * lam)                     # condition number about 20
    H = H0 + np.diag(np.repeat(eps ** 2 * dso ** 2, w.nx * w.nz))
    p_direct = np.linalg.solve(H, b).reshape(w.nh, w.nx, w.nz)
    p, phis = oracle.vp_solve(g, w.vel, geo, dobs, w.nh, eps, dso, 40, lag)
    assert rel_l2(p, p_direct) < 1e-6
    dres = dobs - oracle.model(g, w.vel, geo)
    phi_min = oracle.vp_objective(g, w.vel, geo, p_direct, dres, eps, dso, lag)
    # CG never increases the quadratic objective and stays above its minimum
    assert all(b2 <= a2 * (1 + 1e-12) for a2, b2 in zip(phis, phis[1:]))
    assert min(phis) >= phi_min * (1 - 1e-9)
    assert abs(phis[-1] - phi_min) <= 1e-8 * phis[0]


def test_vp_objective_at_zero_and_eps_zero(vp_case):
    w, g, geo, dobs, H0, b, lag = vp_case
    # at p~ = 0 the objective is half the squared data residual; with eps = 0
    # one CG step moves along b = B~* dres by the exact line-search length
    dres = dobs - oracle.model(g, w.vel, geo)
    p, phis = oracle.vp_solve(g, w.vel, geo, dobs, w.nh, 0.0, synth.dso_weights(w.nh), 1, lag)
    assert phis[0] == pytest.approx(0.5 * float(np.sum(dres ** 2)), rel=1e-14)
    alpha = float(b @ b) / float(b @ (H0 @ b))
    assert rel_l2(p.ravel(), alpha * b) < 1e-10
    assert phis[1] == pytest.approx(phis[0] - 0.5 * alpha * float(b @ b), rel=1e-9)


# ---------------------------------------------------------------------------
# Extended Born with time lags (the time-lag extension of Section 2)
# ---------------------------------------------------------------------------

def test_dot_born_time_lag(small):
    # lags 2kL reach past both ends of the record (nt 120, K 2, L 7: up to 28
    # steps), so dropped terms are exercised too
    w, g, geo = small
    rng = np.random.default_rng(21)
    pt = rng.standard_normal((5, w.nx, w.nz))
    d = rng.standard_normal((w.nshots, w.nrec, w.nt))
    lhs = np.sum(oracle.born_ext_tau_fwd(g, w.vel, geo, pt, 7) * d)
    rhs = np.sum(pt * oracle.born_ext_tau_adj(g, w.vel, geo, d, 5, 7))
    assert dot_err(lhs, rhs) < 1e-10


def test_time_lag_zero_lag_is_born(small):
    # one lag (K = 0): the Born operator of the same perturbation, forward and adjoint
    w, g, geo = small
    rng = np.random.default_rng(22)
    dv = rng.standard_normal((w.nx, w.nz))
    dv_pad = np.zeros((w.nx + 2 * w.nb, w.nz + 2 * w.nb))
    dv_pad[w.nb:w.nb + w.nx, w.nb:w.nb + w.nz] = dv
    fwd = oracle.born_ext_tau_fwd(g, w.vel, geo, dv[None], 3)
    assert rel_l2(fwd, oracle.born(g, w.vel, geo, dv_pad)) < 1e-12
    d = rng.standard_normal((w.nshots, w.nrec, w.nt))
    adj = oracle.born_ext_tau_adj(g, w.vel, geo, d, 1, 3)[0]
    ref = oracle.born_adjoint(g, w.vel, geo, d)[w.nb:w.nb + w.nx, w.nb:w.nb + w.nz]
    assert rel_l2(adj, ref) < 1e-12


@pytest.mark.parametrize("lag", [1, 3])
def test_time_lag_positive_lag_is_a_delay(small, lag):
    # p~ only at lag k = +1: the scattering source of equation n is c T2u_{n-2L},
    # i.e. the zero-lag source delayed by 2L steps, and the recursion is
    # shift-invariant in time, so the data are the zero-lag data delayed by 2L
    w, g, geo = small
    rng = np.random.default_rng(23)
    dv = rng.standard_normal((w.nx, w.nz))
    p1 = np.zeros((3, w.nx, w.nz))
    p1[2] = dv
    d1 = oracle.born_ext_tau_fwd(g, w.vel, geo, p1, lag)
    d0 = oracle.born_ext_tau_fwd(g, w.vel, geo, dv[None], lag)
    sh = 2 * lag
    assert np.abs(d0).max() > 0
    assert np.all(d1[:, :, :sh] == 0)
    assert rel_l2(d1[:, :, sh:], d0[:, :, :-sh]) < 1e-13
