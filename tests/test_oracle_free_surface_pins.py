"""Pins of the oracle's free surface (Grid.free_surface in oracle/fd.py): the
pressure vanishes on the model's first row and the rows above hold the field
mirrored with opposite sign.

* Image source, exact: a run with the free surface equals, below the surface,
  a run without it on the grid mirrored about the surface row, driven by the
  source and its image of opposite sign (velocity and taper mirrored too).
* Analytic: in a homogeneous medium the response is G(r) - G(r'), with r' the
  distance to the image source (the 2D Green's function, within 1e-2).
* Reciprocity, the Born, extended-Born and time-lag dot-product tests, and
  the velocity gradient against central differences, all with the free
  surface on.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from _helpers import oracle_problem, rel_l2
from test_oracle_pins import analytic_green_2d, _homogeneous


def _fs(g):
    return oracle.Grid(g.nz, g.nx, g.nb, g.nt, g.dz, g.dx, g.dt, g.sponge_alpha, True)


def test_free_surface_equals_mirrored_image_source():
    w = synth.tiny(nz=26, nx=34, nb=8, nt=220, nshots=1, seed=5)
    nz, nx, nb = w.nz, w.nx, w.nb
    src = (6, 15)
    rec = np.array([[1, 3], [2, 20], [5, 9], [17, 30]])          # (iz, ix)
    wav = synth.ricker(w.nt, w.dt, 25.0)[None]
    g = oracle.Grid(nz, nx, nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha, True)
    geo = oracle.Geometry(np.array([src[0]]), np.array([src[1]]), rec[None, :, 0], rec[None, :, 1], wav)
    d_fs = oracle.model(g, w.vel, geo)[0]
    # mirrored grid: 2 nz - 1 rows, the surface row in the middle
    c = nz - 1
    vel2 = np.concatenate([w.vel[:, :0:-1], w.vel], axis=1)
    g2 = oracle.Grid(2 * nz - 1, nx, nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
    both = []
    for iz, sign in ((c + src[0], 1.0), (c - src[0], -1.0)):
        geo2 = oracle.Geometry(np.array([iz]), np.array([src[1]]), rec[None, :, 0] + c, rec[None, :, 1], sign * wav)
        both.append(oracle.model(g2, vel2, geo2)[0])
    d_img = both[0] + both[1]
    assert np.abs(d_fs).max() > 0
    assert rel_l2(d_fs, d_img) < 1e-12


def test_free_surface_homogeneous_matches_image_green_function():
    # 10 Hz Ricker, 2000 m/s, 10 m grid; source 150 m below the surface, image
    # 150 m above it; the window ends before the absorbing strips reflect
    c, dx, dt, nt, f = 2000.0, 10.0, 1e-3, 600, 10.0
    src = (15, 100)
    recs = [(10, 140), (40, 128), (3, 100)]
    g, vel, geo = _homogeneous(150, 201, 20, nt, dx, dt, c, src, recs, f)
    d = oracle.model(_fs(g), vel, geo)[0]
    t = np.arange(nt) * dt
    for k, (iz, ix) in enumerate(recs):
        r1 = dx * math.hypot(iz - src[0], ix - src[1])
        r2 = dx * math.hypot(iz + src[0], ix - src[1])
        ref = analytic_green_2d(r1, c, t, f) - analytic_green_2d(r2, c, t, f)
        assert rel_l2(d[k], ref) < 1e-2, k


def test_free_surface_row_records_zero():
    w = synth.tiny(nz=20, nx=24, nb=6, nt=120, nshots=1)
    g, geo = oracle_problem(w)
    geo = oracle.Geometry(geo.src_iz, geo.src_ix, np.zeros_like(geo.rec_iz), geo.rec_ix, geo.wavelet)
    assert np.abs(oracle.model(g, w.vel, geo)).max() > 0
    assert np.abs(oracle.model(_fs(g), w.vel, geo)).max() == 0.0


def test_free_surface_needs_four_strip_rows():
    w = synth.tiny(nz=12, nx=12, nb=3, nt=20, nshots=1)
    g, geo = oracle_problem(w)
    with pytest.raises(ValueError):
        oracle.model(_fs(g), w.vel, geo)


def test_free_surface_reciprocity():
    w = synth.tiny(nz=30, nx=40, nb=10, nt=250, nshots=1)
    g, _ = oracle_problem(w)
    g = _fs(g)
    A, B = (2, 6), (21, 33)
    wav = synth.ricker(w.nt, w.dt, 25.0)[None]

    def shot(s, r):
        geo = oracle.Geometry(np.array([s[0]]), np.array([s[1]]), np.array([[r[0]]]), np.array([[r[1]]]), wav)
        return oracle.model(g, w.vel, geo)[0, 0]
    ab, ba = shot(A, B), shot(B, A)
    assert np.max(np.abs(ab)) > 0
    assert rel_l2(ab, ba) < 1e-12


@pytest.fixture(scope="module")
def fs_small():
    w = synth.tiny(nz=20, nx=28, nb=6, nt=120, nshots=2, nh=5)
    g, geo = oracle_problem(w)
    return w, _fs(g), geo


def test_free_surface_dot_born(fs_small):
    w, g, geo = fs_small
    rng = np.random.default_rng(3)
    dv = rng.standard_normal((w.nx + 2 * w.nb, w.nz + 2 * w.nb))
    d = rng.standard_normal((geo.nshots, w.nrec, w.nt))
    lhs = float(np.sum(oracle.born(g, w.vel, geo, dv) * d))
    rhs = float(np.sum(dv * oracle.born_adjoint(g, w.vel, geo, d)))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))


def test_free_surface_dot_born_extended(fs_small):
    w, g, geo = fs_small
    rng = np.random.default_rng(4)
    p = rng.standard_normal((w.nh, w.nx, w.nz))
    d = rng.standard_normal((geo.nshots, w.nrec, w.nt))
    lhs = float(np.sum(oracle.born_ext_fwd(g, w.vel, geo, p) * d))
    rhs = float(np.sum(p * oracle.born_ext_adj(g, w.vel, geo, d, w.nh)))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))


def test_free_surface_dot_born_time_lag(fs_small):
    w, g, geo = fs_small
    rng = np.random.default_rng(6)
    p = rng.standard_normal((5, w.nx, w.nz))
    d = rng.standard_normal((geo.nshots, w.nrec, w.nt))
    lhs = float(np.sum(oracle.born_ext_tau_fwd(g, w.vel, geo, p, 4) * d))
    rhs = float(np.sum(p * oracle.born_ext_tau_adj(g, w.vel, geo, d, 5, 4)))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))


def test_free_surface_gradient_central_difference():
    w = synth.tiny(nz=16, nx=22, nb=5, nt=110, nshots=2, nh=5, seed=21)
    g, geo = oracle_problem(w)
    g = _fs(g)
    true = w.vel + 80.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 22, 30.0)
    dobs = oracle.model(g, true, geo)
    pt = 0.05 * np.random.default_rng(23).standard_normal((w.nh, w.nx, w.nz))
    dso, eps = synth.dso_weights(w.nh), 1e-3
    _, gv, _ = oracle.gradient(g, w.vel, geo, pt, dobs, eps, dso)
    dm = synth.gaussian_perturbation(w.nz, w.nx, w.dx, 101, 30.0)
    t = 0.1
    fp = oracle.objective(g, w.vel + t * dm, geo, pt, dobs, eps, dso)
    fm = oracle.objective(g, w.vel - t * dm, geo, pt, dobs, eps, dso)
    fd = (fp - fm) / (2 * t)
    an = float(np.sum(gv * dm))
    assert abs(fd - an) / abs(an) < 1e-6, (fd, an)
