"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the method's arithmetic: it only draws velocity
models, wavelets, acquisition geometries and perturbations.  Both the GPU path
and the FP64 oracle receive exactly these arrays as inputs.

The paper's velocity models and datasets (Marmousi2, BP 2004, the Seiscope
syncline, the salt models of Sections 3-7) are not available here; the
generators below stand in for them with the same kind of structure, sizes and
value ranges:

* :func:`smooth_random_velocity` -- Gaussian-filtered white noise mapped
  affinely onto [vmin, vmax] (the smooth heterogeneous media of the tests).
* :func:`marmousi_like` -- 12 dipping, undulating layers from 1500 m/s water to
  4700 m/s, three normal faults and a +-5 % smooth perturbation, standing in for
  the reflection-dominated Marmousi2 benchmark of Section 3.
* :func:`ricker` -- a Ricker wavelet (the paper uses band-limited wavelets,
  Sections 3-7).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter


# ----------------------------------------------------------------------------
# Wavelet
# ----------------------------------------------------------------------------

def ricker_value(t, f_peak: float, t0: float | None = None):
    """Ricker wavelet (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0, t0 = 1.5/f."""
    if t0 is None:
        t0 = 1.5 / f_peak
    a = (math.pi * f_peak * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker(nt: int, dt: float, f_peak: float, t0: float | None = None) -> np.ndarray:
    return ricker_value(np.arange(nt) * dt, f_peak, t0)


# ----------------------------------------------------------------------------
# Velocity models ([nx][nz], z fastest, m/s)
# ----------------------------------------------------------------------------

def smooth_random_field(nz: int, nx: int, sigma_cells: float, seed: int) -> np.ndarray:
    """N(0,1) noise smoothed by a Gaussian of sigma_cells (reflecting edges), [nx][nz]."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nz, nx))
    a = gaussian_filter(a, sigma=sigma_cells, mode="reflect")
    return np.ascontiguousarray(a.T)


def smooth_random_velocity(nz: int, nx: int, dx: float, seed: int,
                           vmin: float = 1500.0, vmax: float = 3500.0,
                           corr_len: float = 300.0) -> np.ndarray:
    a = smooth_random_field(nz, nx, corr_len / dx, seed)
    lo, hi = a.min(), a.max()
    return vmin + (a - lo) * (vmax - vmin) / (hi - lo)


def marmousi_like(nz: int, nx: int, dx: float, seed: int = 2206,
                  vmin: float = 1500.0, vmax: float = 4700.0) -> np.ndarray:
    """Layered, faulted stand-in for Marmousi2, [nx][nz]."""
    rng = np.random.default_rng(seed)
    nl = 12
    depth = nz * dx
    width = nx * dx
    x = np.arange(nx) * dx
    z = np.arange(nz) * dx
    # layer velocities: jittered linspace, layer 0 is water
    base = np.linspace(vmin, vmax, nl)
    jit = rng.uniform(-0.3, 0.3, nl) * (vmax - vmin) / nl
    jit[0] = 0.0
    vlay = np.clip(base + jit, vmin, vmax)
    vlay[0] = vmin
    # interface k (top of layer k), k = 1..nl-1
    zbar = np.linspace(0.08 * depth, 0.92 * depth, nl - 1)
    theta = np.deg2rad(rng.uniform(-8, 8, nl - 1))
    amp = rng.uniform(0.0, 40.0, nl - 1)
    lam = rng.uniform(3000.0, 8000.0, nl - 1)
    phi = rng.uniform(0.0, 2 * np.pi, nl - 1)

    def interfaces(xx):
        return zbar[:, None] + np.tan(theta)[:, None] * (xx[None, :] - width / 2) \
            + amp[:, None] * np.sin(2 * np.pi * xx[None, :] / lam[:, None] + phi[:, None])

    # faults: a straight plane through (xf, 0) dipping at dip; the hanging wall
    # (right of the plane) is shifted down by the throw
    nf = 3
    xf = rng.uniform(0.2 * width, 0.8 * width, nf)
    dip = np.deg2rad(rng.uniform(60, 80, nf))
    throw = rng.uniform(50.0, 200.0, nf)
    X, Z = np.meshgrid(x, z, indexing="ij")           # [nx][nz]
    zshift = np.zeros_like(X)
    for f in range(nf):
        plane_x = xf[f] + Z / np.tan(dip[f])
        zshift -= np.where(X > plane_x, throw[f], 0.0)
    zeff = Z + zshift
    ifc = interfaces(x)                                # [nl-1][nx]
    layer = np.zeros(X.shape, dtype=np.int64)
    for k in range(nl - 1):
        layer += (zeff > ifc[k][:, None]).astype(np.int64)
    vel = vlay[layer]
    # water layer stays flat and unfaulted
    vel[Z < zbar[0] * 0.5] = vmin
    s = smooth_random_field(nz, nx, 200.0 / dx, seed + 1)
    s = s / np.max(np.abs(s))
    vel = vel * (1.0 + 0.05 * s)
    return np.clip(vel, vmin, vmax)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    """One modeling problem: grid, velocity and acquisition (model-grid indices)."""
    name: str
    nz: int
    nx: int
    nb: int
    nt: int
    dz: float
    dx: float
    dt: float
    vel: np.ndarray               # [nx][nz] float64
    src_iz: np.ndarray            # [ns] int32
    src_ix: np.ndarray            # [ns] int32
    rec_iz: np.ndarray            # [ns][nr] int32
    rec_ix: np.ndarray            # [ns][nr] int32
    wavelet: np.ndarray           # [ns][nt] float64
    nh: int = 1
    sponge_alpha: float = 0.3
    extra: dict = field(default_factory=dict)

    @property
    def nshots(self):
        return int(self.src_iz.shape[0])

    @property
    def nrec(self):
        return int(self.rec_ix.shape[1])

    @property
    def padded_cells(self):
        return (self.nz + 2 * self.nb) * (self.nx + 2 * self.nb)

    def subset(self, shots):
        shots = np.asarray(shots)
        return Workload(self.name, self.nz, self.nx, self.nb, self.nt, self.dz, self.dx, self.dt,
                        self.vel, self.src_iz[shots], self.src_ix[shots], self.rec_iz[shots],
                        self.rec_ix[shots], self.wavelet[shots], self.nh, self.sponge_alpha,
                        dict(self.extra))


def surface_line(ns: int, src_ix, nx: int, iz: int = 2, nt: int = 1000, dt: float = 1e-3,
                 f_peak: float = 10.0, rec_ix=None):
    """Sources at (iz, src_ix[s]); receivers at depth iz on every listed column."""
    src_ix = np.asarray(src_ix, dtype=np.int32)
    if rec_ix is None:
        rec_ix = np.arange(nx, dtype=np.int32)
    rec_ix = np.asarray(rec_ix, dtype=np.int32)
    nr = rec_ix.shape[0]
    return dict(src_iz=np.full(ns, iz, dtype=np.int32), src_ix=src_ix,
                rec_iz=np.full((ns, nr), iz, dtype=np.int32),
                rec_ix=np.tile(rec_ix, (ns, 1)).astype(np.int32),
                wavelet=np.tile(ricker(nt, dt, f_peak), (ns, 1)))


def plain_small(seed: int = 1234) -> Workload:
    """100 x 200 grid, 10 m, 40-cell sponge, smooth random 1500-3500 m/s (300 m
    correlation), one 10 Hz Ricker shot at (20 m, 1000 m), 200 receivers at
    20 m depth, dt = 1 ms, nt = 1500, 11 subsurface offsets."""
    nz, nx, dx = 100, 200, 10.0
    vel = smooth_random_velocity(nz, nx, dx, seed, 1500.0, 3500.0, 300.0)
    geo = surface_line(1, [100], nx, iz=2, nt=1500, dt=1e-3, f_peak=10.0)
    return Workload("plain-100x200", nz, nx, 40, 1500, dx, dx, 1e-3, vel, nh=11, **geo)


def marmousi_set(nshots: int = 100, shot_step: int = 17) -> Workload:
    """300 x 1700 Marmousi-like grid, 10 m, 60-cell sponge, shots every 170 m at
    20 m depth, 1700 receivers every 10 m, 8 Hz Ricker, dt = 0.8 ms, nt = 5000,
    61 subsurface offsets."""
    nz, nx, dx = 300, 1700, 10.0
    vel = marmousi_like(nz, nx, dx, 2206)
    src = (np.arange(nshots) * shot_step) % nx
    geo = surface_line(nshots, src, nx, iz=2, nt=5000, dt=8e-4, f_peak=8.0)
    return Workload("marmousi-300x1700", nz, nx, 60, 5000, dx, dx, 8e-4, vel, nh=61, **geo)


def tiny(nz=24, nx=32, nb=8, nt=160, dx=10.0, dt=1e-3, nshots=2, nrec=None, seed=7,
         f_peak=25.0, vmin=1500.0, vmax=2500.0, nh=5, rec_iz=2, src_iz=2) -> Workload:
    """Small heterogeneous problem for fast oracle pins."""
    vel = smooth_random_velocity(nz, nx, dx, seed, vmin, vmax, 60.0)
    rng = np.random.default_rng(seed + 100)
    src = rng.integers(2, nx - 2, nshots)
    rec = np.arange(0, nx, max(1, nx // (nrec or nx)))[: (nrec or nx)]
    geo = surface_line(nshots, src, nx, iz=rec_iz, nt=nt, dt=dt, f_peak=f_peak, rec_ix=rec)
    geo["src_iz"][:] = src_iz
    return Workload(f"tiny-{nz}x{nx}", nz, nx, nb, nt, dx, dx, dt, vel, nh=nh, **geo)


def gaussian_perturbation(nz: int, nx: int, dx: float, seed: int, sigma_m: float = 100.0) -> np.ndarray:
    """Smooth field scaled to max |xi| = 1 (seeded), [nx][nz]."""
    a = smooth_random_field(nz, nx, sigma_m / dx, seed)
    return a / np.max(np.abs(a))


def random_ptilde(nh: int, nz: int, nx: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nh, nx, nz))


def dso_weights(nh: int) -> np.ndarray:
    """Default DSO weights sqrt(ih^2 + 1): |h| made invertible at h = 0."""
    H = (nh - 1) // 2
    ih = np.arange(-H, H + 1, dtype=np.float64)
    return np.sqrt(ih ** 2 + 1.0)


def batch_set(nshots: int = 256, seed: int = 2362, nt_range=(3000, 6000), dt: float = 8e-4,
              sizes=((200, 600), (300, 1700), (500, 2500)), nb: int = 40, dx: float = 10.0) -> list:
    """Shots of uneven grids: each shot is its own job (grid drawn uniformly from
    `sizes`, smooth random 1500-4500 m/s model of that size with 300 m
    correlation, Ricker peak U(6, 12) Hz, nt uniform in nt_range, source at a
    random column 20 m deep, receivers on every column at 20 m)."""
    rng = np.random.default_rng(seed)
    models = [smooth_random_velocity(nz, nx, dx, seed + 1 + i, 1500.0, 4500.0, 300.0)
              for i, (nz, nx) in enumerate(sizes)]
    jobs = []
    for s in range(nshots):
        k = int(rng.integers(len(sizes)))
        nz, nx = sizes[k]
        nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
        f = float(rng.uniform(6.0, 12.0))
        ix = int(rng.integers(0, nx))
        geo = surface_line(1, [ix], nx, iz=2, nt=nt, dt=dt, f_peak=f)
        jobs.append(Workload(f"batch-{nz}x{nx}", nz, nx, nb, nt, dx, dx, dt, models[k], extra={"size": k}, **geo))
    return jobs


@dataclass
class ServeRequestSpec:
    """One request of a serving replay (host-side description only)."""
    arrival: float                # seconds after the replay starts
    kind: str                     # model | born_fwd | born_adj | gradient
    model: int                    # index into the resident model pool
    src_ix: np.ndarray            # [nshots] source columns (20 m deep)
    nt: int
    f_peak: float
    seed: int                     # seeds this request's random inputs


@dataclass
class ServeMix:
    pool: list                    # [(nz, nx, vel [nx][nz] float64)]
    requests: list                # [ServeRequestSpec], sorted by arrival
    nb: int
    dx: float
    dt: float
    nh: int


def serve_mix(nreq: int = 24, seed: int = 42, rate: float = 20.0, npool: int = 6,
              nz_choices=tuple(range(200, 601, 100)), nx_choices=tuple(range(600, 3001, 200)),
              shots=(1, 32), nt_choices=tuple(range(2000, 6001, 500)), dt: float = 8e-4, dx: float = 10.0,
              nb: int = 40, nh: int = 11,
              mix=(("model", 0.4), ("born_fwd", 0.15), ("born_adj", 0.15), ("gradient", 0.3)),
              velocities: bool = True) -> ServeMix:
    """Seeded Poisson request stream over a pool of resident velocity models.

    Inter-arrival times are exponential with mean 1/rate.  The pool holds
    `npool` smooth random 1500-4500 m/s models (300 m correlation) whose grid
    sizes are drawn uniformly from the nz/nx choices; each request picks a
    pool model uniformly, a kind from `mix`, a shot count uniform in `shots`
    (sources at distinct random columns), nt from `nt_choices` and a Ricker
    peak U(6, 12) Hz.  Receivers sit on every column at 20 m depth.  Requests
    are drawn one after the other, so a shorter stream is a prefix of a longer
    one with the same seed.  velocities=False leaves the pool's velocity
    arrays out (None): the request stream is the same."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(npool):
        nz = int(rng.choice(nz_choices))
        nx = int(rng.choice(nx_choices))
        v = smooth_random_velocity(nz, nx, dx, seed + 1 + i, 1500.0, 4500.0, 300.0) if velocities else None
        pool.append((nz, nx, v))
    kinds = [k for k, _ in mix]
    probs = np.array([p for _, p in mix], dtype=np.float64)
    probs /= probs.sum()
    reqs = []
    t_now = 0.0
    for r in range(nreq):
        t_now += float(rng.exponential(1.0 / rate))
        kind = str(rng.choice(kinds, p=probs))
        m = int(rng.integers(npool))
        nx = pool[m][1]
        ns = int(rng.integers(shots[0], shots[1] + 1))
        src = np.sort(rng.choice(nx, size=min(ns, nx), replace=False)).astype(np.int32)
        reqs.append(ServeRequestSpec(t_now, kind, m, src, int(rng.choice(nt_choices)),
                                     float(rng.uniform(6.0, 12.0)), seed * 1000 + r))
    return ServeMix(pool, reqs, nb, dx, dt, nh)


def serve_request_inputs(mix: ServeMix, spec: ServeRequestSpec, device: str = "cuda:0", nt_cap: int | None = None):
    """Geometry arrays (host) and seeded random device tensors for one request.

    ptilde ~ 1e-2 N(0, 1) [nh][nx][nz] for Born forward and gradient requests;
    data ~ N(0, 1) [nshots][nx][nt] for Born adjoint requests; observed data
    ~ 1e-3 N(0, 1) and DSO weights sqrt(ih^2 + 1) for gradient requests.
    nt_cap shortens the time axis (parity runs at the full grid sizes)."""
    import torch
    nz, nx, _ = mix.pool[spec.model]
    nt = spec.nt if nt_cap is None else min(spec.nt, nt_cap)
    ns = len(spec.src_ix)
    geo = surface_line(ns, spec.src_ix, nx, iz=2, nt=nt, dt=mix.dt, f_peak=spec.f_peak)
    gen = torch.Generator(device=device)
    gen.manual_seed(spec.seed)
    out = dict(geo, nt=nt)
    out["wavelet"] = torch.tensor(geo["wavelet"], dtype=torch.float32, device=device)
    if spec.kind in ("born_fwd", "gradient"):
        out["ptilde"] = 1e-2 * torch.randn((mix.nh, nx, nz), generator=gen, device=device)
    if spec.kind == "born_adj":
        out["data"] = torch.randn((ns, nx, nt), generator=gen, device=device)
    if spec.kind == "gradient":
        out["dobs"] = 1e-3 * torch.randn((ns, nx, nt), generator=gen, device=device)
        out["dso"] = dso_weights(mix.nh)
    return out
