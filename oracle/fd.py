"""FP64 NumPy oracle: finite-difference modeling, Born and extended Born, FWIME gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring): never called by the GPU
library, shares no code with it.

What is computed follows Section 2 of the paper (eqs. fwime.obj, vp.obj,
fwime.gradient.split, fwime.gradient.born, fwime.gradient.tomo).  The paper
names the physics (acoustic, isotropic, constant-density two-way wave
equation, Cerjan absorbing boundaries on all sides, point sources and
receivers; Sections 2 and 3) but prints no discretization, so the following
readings are made and used everywhere below:

* Grid and layout.  Arrays are indexed ``[x][z]`` (z fastest).  The model grid
  (nz, nx) is surrounded by an absorbing strip of ``nb`` cells on every side;
  the velocity is replicated from the nearest edge cell into the strip
  (operator ``P``, :func:`pad_edge`).  Padded sizes NZ = nz + 2 nb,
  NX = nx + 2 nb.
* Space: the radius-4 (8th-order) central second derivative whose weights come
  from Fornberg's algorithm (:func:`fd_second_derivative_weights`), summed over
  z and x; values outside the padded grid are zero.
* Time: second-order leapfrog.  With D = 1/(v^2 dt^2) and the Cerjan taper g
  (1 inside the model grid), equation n (n = 0 .. nt-2) of the discrete system
  reads  D (u^{n+1}/g - 2 u^n + g u^{n-1}) - L u^n = f^n,  with
  u^{-1} = u^0 = 0, i.e.  u^{n+1} = g (2 u^n - g u^{n-1} + V (L u^n + f^n)),
  V = v^2 dt^2.  All three time blocks of the system matrix are symmetric, so
  the adjoint is the same recursion run backwards in time and
  source-receiver reciprocity holds exactly.
* Taper: g = g_z(iz) g_x(ix), g_1D(k) = exp(-(alpha k / nb)^2) for the cell k
  = 1..nb cells into the strip (Cerjan et al.'s Gaussian profile;
  alpha = 0.3 reproduces their edge value exp(-0.09)).
* Free surface (``Grid.free_surface``; the free-surface-multiples variant of
  the Marmousi2 test in Section 3 models with a free surface at the water
  surface and absorbing boundaries elsewhere, after Robertsson's image-based
  condition): the pressure vanishes on the model's first row (padded row nb),
  and the Laplacian of the rows below reads
  the field mirrored with opposite sign above it (the image method: u(nb - k)
  = -u(nb + k)).  The field at and above the surface row stays zero, so the
  top strip is unused.  The mirrored operator is symmetric on the remaining
  rows, so the adjoint recursion and reciprocity hold as without it.
* Point source: f^n = w(n dt) / (dx dz) at the source cell, so the scheme
  approximates (1/v^2) u_tt - Laplacian u = delta(x) w(t).  Receivers sample
  u^k at their cell, k = 0 .. nt-1 (d^0 = 0).
* Model parameter: velocity (m/s).  The Born scattering source of a velocity
  perturbation dv in equation n is (2 dv / (v^3 dt^2)) T2u_n with
  T2u_n = u^{n+1}/g - 2 u^n + g u^{n-1}  (the exact linearization of D).
* Extension: horizontal subsurface offset h = ih dx, ih in [-H, H], nh = 2H+1,
  symmetric convention.  The extended perturbation p~(z, y, h) lives on the
  model grid; the forward source is
  s_n(z, y+h) += 2 p~(z,y,h) / (v(z,y)^3 dt^2) * T2u_n(z, y-h)
  (terms leaving the padded grid are dropped); at h = 0 this is Born.
* Time-lag extension (the other extension of Section 2, the paper's choice
  in four of its five examples; its discretization is not printed either):
  lag tau_k = k L dt, k in [-K, K], ntau = 2K+1, L a whole number of time
  steps, symmetric convention (source side t - tau, receiver side t + tau).
  The extended perturbation p~(z, y, k) lives on the model grid; the
  scattering source of equation n is
  s_n(z, y) += 2 p~(z,y,k) / (v(z,y)^3 dt^2) * T2u_{n - 2kL}(z, y)
  for 0 <= n - 2kL <= nt - 2 (other terms are dropped); at K = 0 this is Born.
* DSO operator D of eq. fwime.obj: diagonal, weight d_h per offset, supplied
  by the caller.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np


# ----------------------------------------------------------------------------
# Stencil weights, stability limit, taper, padding
# ----------------------------------------------------------------------------

def fd_second_derivative_weights(radius: int = 4) -> list[Fraction]:
    """Weights w_0..w_radius of the central second derivative on a unit grid.

    Fornberg's recursion (Fornberg 1988, "Generation of finite difference
    formulas on arbitrarily spaced grids") over the nodes 0, 1, -1, 2, -2, ...,
    evaluated in exact rationals; the symmetric weight of node +k and -k is
    returned once.
    """
    nodes = [0]
    for k in range(1, radius + 1):
        nodes += [k, -k]
    n = len(nodes)
    m = 2  # derivative order
    c = [[Fraction(0)] * n for _ in range(m + 1)]
    c[0][0] = Fraction(1)
    c1 = Fraction(1)
    c4 = Fraction(nodes[0])
    for i in range(1, n):
        mn = min(i, m)
        c2 = Fraction(1)
        c5 = c4
        c4 = Fraction(nodes[i])
        for j in range(i):
            c3 = Fraction(nodes[i] - nodes[j])
            c2 *= c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[k][i] = c1 * (k * c[k - 1][i - 1] - c5 * c[k][i - 1]) / c2
                c[0][i] = -c1 * c5 * c[0][i - 1] / c2
            for k in range(mn, 0, -1):
                c[k][j] = (c4 * c[k][j] - k * c[k - 1][j]) / c3
            c[0][j] = c4 * c[0][j] / c3
        c1 = c2
    w = [c[2][0]]
    for k in range(1, radius + 1):
        assert c[2][2 * k - 1] == c[2][2 * k]
        w.append(c[2][2 * k - 1])
    return w


_W = [float(x) for x in fd_second_derivative_weights(4)]


def cfl_limit(dz: float, dx: float) -> float:
    """Largest stable v_max * dt for the leapfrog scheme with the radius-4 Laplacian.

    Von Neumann: leapfrog is stable iff V * rho(-L) <= 4, and the symbol of the
    1-D second difference is extreme at the Nyquist wavenumber, where it equals
    (w_0 + 2 sum_k (-1)^k w_k) / d^2.
    """
    nyq = -(_W[0] + 2.0 * sum(((-1) ** k) * _W[k] for k in range(1, 5)))
    return 2.0 / np.sqrt(nyq * (1.0 / dz ** 2 + 1.0 / dx ** 2))


def sponge_profile(n: int, nb: int, alpha: float) -> np.ndarray:
    """Cerjan taper along one padded axis of length n + 2 nb (1 on the model grid)."""
    g = np.ones(n + 2 * nb)
    for i in range(n + 2 * nb):
        if i < nb:
            k = nb - i
        elif i >= nb + n:
            k = i - (nb + n - 1)
        else:
            continue
        g[i] = np.exp(-(alpha * k / nb) ** 2)
    return g


def pad_edge(a: np.ndarray, nb: int) -> np.ndarray:
    """P: replicate the nearest model-grid value into the absorbing strip."""
    return np.pad(a, nb, mode="edge")


def pad_edge_adjoint(ap: np.ndarray, nb: int) -> np.ndarray:
    """P^T: every padded cell adds its value into the model cell it was copied from."""
    NX, NZ = ap.shape
    nx, nz = NX - 2 * nb, NZ - 2 * nb
    out = np.zeros((nx, nz))
    ix = np.clip(np.arange(NX) - nb, 0, nx - 1)
    iz = np.clip(np.arange(NZ) - nb, 0, nz - 1)
    for i in range(NX):
        np.add.at(out[ix[i]], iz, ap[i])
    return out


def laplacian(u: np.ndarray, dz: float, dx: float) -> np.ndarray:
    """Radius-4 Laplacian (d2/dz2 + d2/dx2) with zero values outside the array."""
    NX, NZ = u.shape
    r = 4
    p = np.zeros((NX + 2 * r, NZ + 2 * r))
    p[r:r + NX, r:r + NZ] = u
    out = _W[0] * (1.0 / dz ** 2 + 1.0 / dx ** 2) * u
    for k in range(1, r + 1):
        out = out + (_W[k] / dz ** 2) * (p[r:r + NX, r + k:r + k + NZ] + p[r:r + NX, r - k:r - k + NZ])
        out = out + (_W[k] / dx ** 2) * (p[r + k:r + k + NX, r:r + NZ] + p[r - k:r - k + NX, r:r + NZ])
    return out


# ----------------------------------------------------------------------------
# Problem description
# ----------------------------------------------------------------------------

@dataclass
class Grid:
    """Model grid (unpadded) and time axis."""
    nz: int
    nx: int
    nb: int
    nt: int
    dz: float
    dx: float
    dt: float
    sponge_alpha: float = 0.3
    free_surface: bool = False


@dataclass
class Geometry:
    """Acquisition: model-grid indices of sources and receivers, and wavelets."""
    src_iz: np.ndarray   # [nshots]
    src_ix: np.ndarray   # [nshots]
    rec_iz: np.ndarray   # [nshots][nrec]
    rec_ix: np.ndarray   # [nshots][nrec]
    wavelet: np.ndarray  # [nshots][nt]

    @property
    def nshots(self) -> int:
        return int(len(self.src_iz))


class _Medium:
    """Padded velocity, V = v^2 dt^2 and the taper for one velocity model."""

    def __init__(self, g: Grid, vel: np.ndarray):
        vel = np.asarray(vel, dtype=np.float64)
        assert vel.shape == (g.nx, g.nz)
        self.g = g
        self.vel = vel
        self.vpad = pad_edge(vel, g.nb)
        self.V = self.vpad ** 2 * g.dt ** 2
        gx = sponge_profile(g.nx, g.nb, g.sponge_alpha)
        gz = sponge_profile(g.nz, g.nb, g.sponge_alpha)
        self.gam = np.outer(gx, gz)
        self.shape = self.vpad.shape
        self.fs = bool(g.free_surface)
        if self.fs and g.nb < 4:
            raise ValueError("a free surface needs nb >= 4 (the mirrored stencil rows)")

    def lap(self, u):
        if not self.fs:
            return laplacian(u, self.g.dz, self.g.dx)
        # free surface on the model's first row: zero there, mirrored with
        # opposite sign above it, nothing computed at or above it
        nb = self.g.nb
        m = np.zeros_like(u)
        m[:, nb + 1:] = u[:, nb + 1:]
        for k in range(1, 5):
            m[:, nb - k] = -u[:, nb + k]
        out = laplacian(m, self.g.dz, self.g.dx)
        out[:, :nb + 1] = 0.0
        return out

    def restrict(self, u):
        """With a free surface, the field at and above the surface row is zero."""
        if self.fs:
            u[:, :self.g.nb + 1] = 0.0
        return u

    def forward_record(self, source, rec_x, rec_z, keep=False):
        """Forward solve and sample receivers: returns (data[nrec][nt], history|None)."""
        nt = self.g.nt
        V, gam = self.V, self.gam
        u_prev = np.zeros(self.shape)
        u = np.zeros(self.shape)
        data = np.zeros((len(rec_x), nt))
        hist = [u.copy()] if keep else None
        for n in range(nt - 1):
            f = source(n)
            rhs = self.lap(u) if f is None else self.lap(u) + f
            u_next = self.restrict(gam * (2.0 * u - gam * u_prev + V * rhs))
            u_prev, u = u, u_next
            data[:, n + 1] = u[rec_x, rec_z]
            if keep:
                hist.append(u.copy())
        return data, (np.array(hist) if keep else None)

    def adjoint(self, adj_source):
        """Solve the transposed system backwards in time.

        lambda_{nt-1} = lambda_nt = 0 and, for k = nt-1 .. 1,
        lambda_{k-1} = g (2 lambda_k - g lambda_{k+1} + V (L lambda_k + g^k)),
        where adj_source(k) gives g^k (dense) or None.  lambda_n is the
        multiplier of equation n.  Returns lam[0..nt-1] with lam[nt-1] = 0.
        """
        nt = self.g.nt
        V, gam = self.V, self.gam
        lam = np.zeros((nt,) + self.shape)
        lam_next = np.zeros(self.shape)   # lambda_{k+1}
        cur = np.zeros(self.shape)        # lambda_k
        for k in range(nt - 1, 0, -1):
            s = adj_source(k)
            rhs = self.lap(cur) if s is None else self.lap(cur) + s
            prev = self.restrict(gam * (2.0 * cur - gam * lam_next + V * rhs))
            lam[k - 1] = prev
            lam_next, cur = cur, prev
        return lam

    def t2(self, hist, n):
        """T2u_n = u^{n+1}/g - 2 u^n + g u^{n-1} (u^{-1} = 0), n = 0 .. nt-2."""
        um = hist[n - 1] if n >= 1 else 0.0
        return hist[n + 1] / self.gam - 2.0 * hist[n] + self.gam * um


def _point_source(med: _Medium, geom: Geometry, s: int):
    g = med.g
    px, pz = int(geom.src_ix[s]) + g.nb, int(geom.src_iz[s]) + g.nb
    w = np.asarray(geom.wavelet[s], dtype=np.float64)
    scale = 1.0 / (g.dx * g.dz)

    def source(n):
        f = np.zeros(med.shape)
        f[px, pz] = w[n] * scale
        return f
    return source


def _receivers(med: _Medium, geom: Geometry, s: int):
    nb = med.g.nb
    return (np.asarray(geom.rec_ix[s], dtype=np.int64) + nb,
            np.asarray(geom.rec_iz[s], dtype=np.int64) + nb)


def _receiver_injection(med: _Medium, rx, rz, data_s):
    """R^T: g^k = sum over receivers of d^k_r placed at the receiver cell."""
    def adj_source(k):
        f = np.zeros(med.shape)
        np.add.at(f, (rx, rz), data_s[:, k])
        return f
    return adj_source


def _check(g: Grid, vel: np.ndarray, geom: Geometry):
    vmax = float(np.max(vel))
    if vmax * g.dt > cfl_limit(g.dz, g.dx) * (1 + 1e-12):
        raise ValueError("CFL condition violated")
    for a, n in ((geom.src_iz, g.nz), (geom.src_ix, g.nx), (geom.rec_iz, g.nz), (geom.rec_ix, g.nx)):
        a = np.asarray(a)
        if a.size and (a.min() < 0 or a.max() >= n):
            raise ValueError("geometry outside the model grid")


# ----------------------------------------------------------------------------
# Nonlinear modeling f(m) (eq. fwime.obj, first term)
# ----------------------------------------------------------------------------

def model(g: Grid, vel: np.ndarray, geom: Geometry) -> np.ndarray:
    """d[s][r][k] = u^k at receiver r for the point source of shot s."""
    _check(g, vel, geom)
    med = _Medium(g, vel)
    nrec = np.asarray(geom.rec_ix).shape[1]
    out = np.zeros((geom.nshots, nrec, g.nt))
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        out[s], _ = med.forward_record(_point_source(med, geom, s), rx, rz)
    return out


def model_adjoint_wavelet(g: Grid, vel: np.ndarray, geom: Geometry, data: np.ndarray) -> np.ndarray:
    """Adjoint of wavelet -> data: w~^n = lambda_n(src) / (dx dz), w~^{nt-1} = 0."""
    med = _Medium(g, vel)
    out = np.zeros((geom.nshots, g.nt))
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        lam = med.adjoint(_receiver_injection(med, rx, rz, np.asarray(data[s], dtype=np.float64)))
        px, pz = int(geom.src_ix[s]) + g.nb, int(geom.src_iz[s]) + g.nb
        out[s, :g.nt - 1] = lam[:g.nt - 1, px, pz] / (g.dx * g.dz)
    return out


# ----------------------------------------------------------------------------
# Born modeling B and its adjoint (eq. fwime.gradient.born)
# ----------------------------------------------------------------------------

def born(g: Grid, vel: np.ndarray, geom: Geometry, dvel_pad: np.ndarray) -> np.ndarray:
    """Born data of a velocity perturbation given on the PADDED grid.

    The scattering source of equation n is (2 dv / (v^3 dt^2)) T2u_n.
    """
    med = _Medium(g, vel)
    coef = 2.0 * np.asarray(dvel_pad, dtype=np.float64) / (med.vpad ** 3 * g.dt ** 2)
    nrec = np.asarray(geom.rec_ix).shape[1]
    out = np.zeros((geom.nshots, nrec, g.nt))
    for s in range(geom.nshots):
        _, hist = med.forward_record(_point_source(med, geom, s), *_receivers(med, geom, s), keep=True)
        rx, rz = _receivers(med, geom, s)
        out[s], _ = med.forward_record(lambda n: coef * med.t2(hist, n), rx, rz)
    return out


def born_adjoint(g: Grid, vel: np.ndarray, geom: Geometry, data: np.ndarray) -> np.ndarray:
    """B^T d on the padded grid: sum_n (2 / (v^3 dt^2)) T2u_n lambda_n, summed over shots."""
    med = _Medium(g, vel)
    out = np.zeros(med.shape)
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        _, hist = med.forward_record(_point_source(med, geom, s), rx, rz, keep=True)
        lam = med.adjoint(_receiver_injection(med, rx, rz, np.asarray(data[s], dtype=np.float64)))
        for n in range(g.nt - 1):
            out += med.t2(hist, n) * lam[n]
    return out * 2.0 / (med.vpad ** 3 * g.dt ** 2)


# ----------------------------------------------------------------------------
# Extended Born B~ (horizontal subsurface offsets) and its adjoint
# ----------------------------------------------------------------------------

def _offsets(nh: int) -> np.ndarray:
    if nh < 1 or nh % 2 == 0:
        raise ValueError("nh must be odd and positive")
    H = (nh - 1) // 2
    return np.arange(-H, H + 1)


def _ext_coef(med: _Medium, ptilde: np.ndarray) -> np.ndarray:
    """c(z,y,h) = 2 p~(z,y,h) / (v(z,y)^3 dt^2) on the model grid, [nh][nx][nz]."""
    return 2.0 * np.asarray(ptilde, dtype=np.float64) / (med.vel[None] ** 3 * med.g.dt ** 2)


def _y_range(NX: int, nb: int, nx: int, ih: int):
    """Model columns y whose source side y-h and receiver side y+h stay on the padded grid."""
    y = np.arange(nx)
    yp = y + nb
    ok = (yp - ih >= 0) & (yp - ih < NX) & (yp + ih >= 0) & (yp + ih < NX)
    return y[ok]


def _ext_scatter(med: _Medium, coef: np.ndarray, hs: np.ndarray, field: np.ndarray) -> np.ndarray:
    """s(z, y+h) = sum_h c(z,y,h) field(z, y-h), on the padded grid."""
    g = med.g
    nb = g.nb
    NX = med.shape[0]
    out = np.zeros(med.shape)
    zs = slice(nb, nb + g.nz)
    for i, ih in enumerate(hs):
        y = _y_range(NX, nb, g.nx, ih)
        if y.size == 0:
            continue
        out[y + nb + ih, zs] += coef[i, y, :] * field[y + nb - ih, zs]
    return out


def born_ext_fwd(g: Grid, vel: np.ndarray, geom: Geometry, ptilde: np.ndarray) -> np.ndarray:
    """B~ p~: data of the extended scattering source built from T2u_n."""
    _check(g, vel, geom)
    med = _Medium(g, vel)
    nh = ptilde.shape[0]
    hs = _offsets(nh)
    coef = _ext_coef(med, ptilde)
    nrec = np.asarray(geom.rec_ix).shape[1]
    out = np.zeros((geom.nshots, nrec, g.nt))
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        _, hist = med.forward_record(_point_source(med, geom, s), rx, rz, keep=True)
        out[s], _ = med.forward_record(lambda n: _ext_scatter(med, coef, hs, med.t2(hist, n)), rx, rz)
    return out


def _ext_image(med: _Medium, hs, T2, lam) -> np.ndarray:
    """sum_n T2_n(z, y-h) lam_n(z, y+h) on the model grid, [nh][nx][nz] (no coefficient)."""
    g = med.g
    nb = g.nb
    NX = med.shape[0]
    out = np.zeros((len(hs), g.nx, g.nz))
    zs = slice(nb, nb + g.nz)
    for n in range(g.nt - 1):
        t = T2(n)
        for i, ih in enumerate(hs):
            y = _y_range(NX, nb, g.nx, ih)
            if y.size == 0:
                continue
            out[i, y, :] += t[y + nb - ih, zs] * lam[n][y + nb + ih, zs]
    return out


def born_ext_adj(g: Grid, vel: np.ndarray, geom: Geometry, data: np.ndarray, nh: int) -> np.ndarray:
    """B~^T d: p~(z,y,h) = 2/(v(z,y)^3 dt^2) sum_s sum_n T2u_n(z,y-h) lambda_n(z,y+h)."""
    _check(g, vel, geom)
    med = _Medium(g, vel)
    hs = _offsets(nh)
    acc = np.zeros((nh, g.nx, g.nz))
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        _, hist = med.forward_record(_point_source(med, geom, s), rx, rz, keep=True)
        lam = med.adjoint(_receiver_injection(med, rx, rz, np.asarray(data[s], dtype=np.float64)))
        acc += _ext_image(med, hs, lambda n: med.t2(hist, n), lam)
    return acc * 2.0 / (med.vel[None] ** 3 * g.dt ** 2)


# ----------------------------------------------------------------------------
# Extended Born with time lags and its adjoint
# ----------------------------------------------------------------------------

def _lags(ntau: int) -> np.ndarray:
    if ntau < 1 or ntau % 2 == 0:
        raise ValueError("ntau must be odd and positive")
    K = (ntau - 1) // 2
    return np.arange(-K, K + 1)


def born_ext_tau_fwd(g: Grid, vel: np.ndarray, geom: Geometry, ptau: np.ndarray, lag: int) -> np.ndarray:
    """B~_tau p~: data of the time-lag scattering source.

    The source of equation n is sum_k c(z,y,k) T2u_{n-2kL}(z,y) on the model
    grid, c = 2 p~ / (v^3 dt^2), L = lag (time steps per lag unit); terms whose
    background time falls outside equations 0 .. nt-2 are dropped.
    """
    _check(g, vel, geom)
    if int(lag) < 1:
        raise ValueError("lag must be a positive number of time steps")
    med = _Medium(g, vel)
    ks = _lags(ptau.shape[0])
    coef = _ext_coef(med, ptau)
    nb = g.nb
    zs, ys = slice(nb, nb + g.nz), slice(nb, nb + g.nx)
    nrec = np.asarray(geom.rec_ix).shape[1]
    out = np.zeros((geom.nshots, nrec, g.nt))
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        _, hist = med.forward_record(_point_source(med, geom, s), rx, rz, keep=True)

        def source(n):
            src = np.zeros(med.shape)
            for i, k in enumerate(ks):
                m = n - 2 * int(k) * int(lag)
                if 0 <= m <= g.nt - 2:
                    src[ys, zs] += coef[i] * med.t2(hist, m)[ys, zs]
            return src

        out[s], _ = med.forward_record(source, rx, rz)
    return out


def born_ext_tau_adj(g: Grid, vel: np.ndarray, geom: Geometry, data: np.ndarray, ntau: int, lag: int) -> np.ndarray:
    """B~_tau^T d: p~(z,y,k) = 2/(v^3 dt^2) sum_s sum_n T2u_{n-2kL}(z,y) lambda_n(z,y)."""
    _check(g, vel, geom)
    if int(lag) < 1:
        raise ValueError("lag must be a positive number of time steps")
    med = _Medium(g, vel)
    ks = _lags(ntau)
    nb = g.nb
    zs, ys = slice(nb, nb + g.nz), slice(nb, nb + g.nx)
    acc = np.zeros((ntau, g.nx, g.nz))
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        _, hist = med.forward_record(_point_source(med, geom, s), rx, rz, keep=True)
        lam = med.adjoint(_receiver_injection(med, rx, rz, np.asarray(data[s], dtype=np.float64)))
        for n in range(g.nt - 1):
            for i, k in enumerate(ks):
                m = n - 2 * int(k) * int(lag)
                if 0 <= m <= g.nt - 2:
                    acc[i] += med.t2(hist, m)[ys, zs] * lam[n][ys, zs]
    return acc * 2.0 / (med.vel[None] ** 3 * g.dt ** 2)


# ----------------------------------------------------------------------------
# FWIME objective (eq. fwime.obj at a given p~) and its gradient
# ----------------------------------------------------------------------------

def objective(g: Grid, vel, geom: Geometry, ptilde, dobs, eps: float, dso, lag=None) -> float:
    """Phi = 1/2 || f(m) + B~(m) p~ - d_obs ||^2 + eps^2/2 || D p~ ||^2 (forward operators only);
    B~ extends with subsurface offsets, or with time lags of `lag` steps when lag is given."""
    ext = born_ext_fwd(g, vel, geom, ptilde) if lag is None else born_ext_tau_fwd(g, vel, geom, ptilde, lag)
    r = model(g, vel, geom) + ext - np.asarray(dobs, dtype=np.float64)
    dso = np.asarray(dso, dtype=np.float64)
    return 0.5 * float(np.sum(r * r)) + 0.5 * eps ** 2 * float(np.sum((dso[:, None, None] * ptilde) ** 2))


def gradient(g: Grid, vel, geom: Geometry, ptilde, dobs, eps: float, dso, lag=None):
    """Objective and gradients of eq. fwime.obj at a fixed p~.

    With p~ held fixed (at the variable-projection optimum the partial
    derivative in p~ vanishes, so this is the total derivative there), the
    velocity gradient is B^T r + T^T r (eqs. fwime.gradient.split,
    fwime.gradient.born, fwime.gradient.tomo, without the spline operator):

      u = M^{-1} f,  du~ = M^{-1} s(p~),  r = R(u + du~) - d_obs,
      lambda = M^{-T} R^T r.
      Born part:  g_B = sum_n (2/(v^3 dt^2)) T2u_n lambda_n.
      Tomographic part (derivative of B~(m) p~ in m), three terms:
        g_1 = sum_n (2/(v^3 dt^2)) T2du~_n lambda_n          (M depends on v)
        g_2 = sum_n (2/(v^3 dt^2)) T2u_n rho_n                (u depends on v)
              with e_n(z,x) = sum_h c(z,x+h,h) lambda_n(z,x+2h),
              nu^k = e_{k-1}/g - 2 e_k + g e_{k+1},  rho = M^{-T} nu
        g_3 = -sum_h sum_n (6 p~/(v^4 dt^2)) T2u_n(z,y-h) lambda_n(z,y+h)
                                                              (coefficient depends on v)
      grad_vel = P^T (g_B + g_1 + g_2) + g_3,
      grad_p~  = B~^T r + eps^2 d_h^2 p~.

    With time lags (lag = L steps) the scattering source of equation n is
    sum_k c_k T2u_{n-2kL}, so e_m = sum_k c_k lambda_{m+2kL} and g_3 takes
    sum_k sum_n T2u_{n-2kL} lambda_n in place of the offset image; the rest
    is unchanged.
    """
    _check(g, vel, geom)
    med = _Medium(g, vel)
    ptilde = np.asarray(ptilde, dtype=np.float64)
    dso = np.asarray(dso, dtype=np.float64)
    nh = ptilde.shape[0]
    hs = _offsets(nh) if lag is None else _lags(nh)
    if lag is not None and int(lag) < 1:
        raise ValueError("lag must be a positive number of time steps")
    coef = _ext_coef(med, ptilde)
    nb, nt = g.nb, g.nt
    NX = med.shape[0]
    zs, ys = slice(nb, nb + g.nz), slice(nb, nb + g.nx)

    def scatter(n, hu):
        if lag is None:
            return _ext_scatter(med, coef, hs, med.t2(hu, n))
        src = np.zeros(med.shape)
        for i, k in enumerate(hs):
            m = n - 2 * int(k) * int(lag)
            if 0 <= m <= nt - 2:
                src[ys, zs] += coef[i] * med.t2(hu, m)[ys, zs]
        return src

    gpad = np.zeros(med.shape)               # g_B + g_1 + g_2 before the 2/(v^3 dt^2) factor
    img = np.zeros((nh, g.nx, g.nz))         # sum_n T2u(y-h) lambda(y+h)
    misfit = 0.0
    for s in range(geom.nshots):
        rx, rz = _receivers(med, geom, s)
        d_u, hu = med.forward_record(_point_source(med, geom, s), rx, rz, keep=True)
        d_du, hdu = med.forward_record(lambda n: scatter(n, hu), rx, rz, keep=True)
        r = d_u + d_du - np.asarray(dobs[s], dtype=np.float64)
        misfit += 0.5 * float(np.sum(r * r))
        lam = med.adjoint(_receiver_injection(med, rx, rz, r))

        # spreading transpose e_n and the adjoint field rho it drives
        e = np.zeros((nt + 1,) + med.shape)   # e[n] for n = 0..nt-2, zero beyond
        for n in range(nt - 1):
            for i, ih in enumerate(hs):
                if lag is not None:
                    m = n + 2 * int(ih) * int(lag)
                    if 0 <= m <= nt - 2:
                        e[n][ys, zs] += coef[i] * lam[m][ys, zs]
                    continue
                y = _y_range(NX, nb, g.nx, ih)
                if y.size == 0:
                    continue
                e[n][y + nb - ih, zs] += coef[i, y, :] * lam[n][y + nb + ih, zs]

        def nu(k):
            em = e[k - 1] if k >= 1 else 0.0
            return em / med.gam - 2.0 * e[k] + med.gam * e[k + 1]
        rho = med.adjoint(nu)

        for n in range(nt - 1):
            t2u = med.t2(hu, n)
            gpad += (t2u + med.t2(hdu, n)) * lam[n] + t2u * rho[n]
        if lag is None:
            img += _ext_image(med, hs, lambda n: med.t2(hu, n), lam)
        else:
            for n in range(nt - 1):
                for i, k in enumerate(hs):
                    m = n - 2 * int(k) * int(lag)
                    if 0 <= m <= nt - 2:
                        img[i] += med.t2(hu, m)[ys, zs] * lam[n][ys, zs]

    gpad *= 2.0 / (med.vpad ** 3 * g.dt ** 2)
    img_scaled = img * 2.0 / (med.vel[None] ** 3 * g.dt ** 2)          # B~^T r
    g3 = -np.sum(ptilde * img, axis=0) * 6.0 / (med.vel ** 4 * g.dt ** 2)
    grad_vel = pad_edge_adjoint(gpad, nb) + g3
    grad_pt = img_scaled + eps ** 2 * (dso ** 2)[:, None, None] * ptilde
    obj = misfit + 0.5 * eps ** 2 * float(np.sum((dso[:, None, None] * ptilde) ** 2))
    return obj, grad_vel, grad_pt


# ----------------------------------------------------------------------------
# Variable-projection step (eqs. vp.obj, pert.opt, vp.pseudo.inv)
# ----------------------------------------------------------------------------

def _ext_pair(nh: int, lag):
    """B~ and B~^T of the chosen extension: subsurface offsets (lag None) or
    time lags with lag step `lag` (nh lags)."""
    if lag is None:
        return (lambda g, vel, geom, x: born_ext_fwd(g, vel, geom, x),
                lambda g, vel, geom, d: born_ext_adj(g, vel, geom, d, nh))
    return (lambda g, vel, geom, x: born_ext_tau_fwd(g, vel, geom, x, lag),
            lambda g, vel, geom, d: born_ext_tau_adj(g, vel, geom, d, nh, lag))


def vp_objective(g: Grid, vel, geom: Geometry, ptilde, dres, eps: float, dso, lag=None) -> float:
    """Phi_eps,m(p~) = 1/2 || B~ p~ - dres ||^2 + eps^2/2 || D p~ ||^2, dres = d_obs - f(m) (eq. vp.obj).

    lag None: subsurface offsets; otherwise time lags with that lag step."""
    fwd, _ = _ext_pair(np.asarray(ptilde).shape[0], lag)
    r = fwd(g, vel, geom, ptilde) - np.asarray(dres, dtype=np.float64)
    dso = np.asarray(dso, dtype=np.float64)
    return 0.5 * float(np.sum(r * r)) + 0.5 * eps ** 2 * float(np.sum((dso[:, None, None] * ptilde) ** 2))


def vp_solve(g: Grid, vel, geom: Geometry, dobs, nh: int, eps: float, dso, niter: int, lag=None):
    """Variable-projection step by linear conjugate gradient.

    The minimizer of eq. vp.obj solves the normal equation
    (B~* B~ + eps^2 D* D) p~ = B~* (d_obs - f(m)) (eqs. pert.opt and
    vp.pseudo.inv); Section 2 minimizes it with linear conjugate gradient.
    Here: plain CG on that symmetric system from p~ = 0, niter iterations
    (stopping early only if the search direction has zero curvature).
    Returns p~ and Phi_eps,m at p~_0 = 0, p~_1, ..., each evaluated from its
    definition (one extra application of B~ per iterate).  B~ is extended
    with subsurface offsets (lag None) or with nh time lags of step `lag`.
    """
    fwd, adj = _ext_pair(nh, lag)
    dres = np.asarray(dobs, dtype=np.float64) - model(g, vel, geom)
    d2 = (eps * np.asarray(dso, dtype=np.float64)) ** 2

    def normal(x):
        return adj(g, vel, geom, fwd(g, vel, geom, x)) + d2[:, None, None] * x

    b = adj(g, vel, geom, dres)
    p = np.zeros_like(b)
    r = b.copy()
    s = r.copy()
    rr = float(np.sum(r * r))
    phis = [0.5 * float(np.sum(dres * dres))]
    for _ in range(niter):
        q = normal(s)
        curv = float(np.sum(s * q))
        if curv <= 0.0:
            break
        alpha = rr / curv
        p = p + alpha * s
        r = r - alpha * q
        rr_new = float(np.sum(r * r))
        s = r + (rr_new / rr) * s
        rr = rr_new
        phis.append(vp_objective(g, vel, geom, p, dres, eps, dso, lag))
    return p, phis
