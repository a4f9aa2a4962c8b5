"""Shared test helpers: conversions from synth workloads, error metrics."""
import numpy as np

import oracle
import synth


def oracle_problem(w: synth.Workload, alpha=None):
    g = oracle.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt,
                    w.sponge_alpha if alpha is None else alpha)
    geo = oracle.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix, w.wavelet)
    return g, geo


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dot_err(a, b):
    return abs(a - b) / max(abs(a), abs(b))


def gpu_problem(w, dev="cuda:0"):
    """synth workload -> (Grid, vel tensor, Geometry) for the HIP library."""
    import torch
    import paper_2206_02362_amd as fw
    grid = fw.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
    vel = torch.tensor(w.vel, dtype=torch.float32, device=dev)
    wav = torch.tensor(w.wavelet, dtype=torch.float32, device=dev)
    geo = fw.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix, wav)
    return grid, vel, geo


def oracle_problem_f32(w):
    """Oracle inputs rounded to float32 first, so both sides see identical inputs."""
    import oracle
    import synth
    w32 = synth.Workload(w.name, w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt,
                         w.vel.astype(np.float32).astype(np.float64), w.src_iz, w.src_ix, w.rec_iz, w.rec_ix,
                         w.wavelet.astype(np.float32).astype(np.float64), w.nh, w.sponge_alpha)
    g = oracle.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
    geo = oracle.Geometry(w32.src_iz, w32.src_ix, w32.rec_iz, w32.rec_ix, w32.wavelet)
    return g, geo, w32.vel


def serve_setup(mix, server, dev="cuda:0", nt_cap=None):
    """Register the pool's models on `server` and build one Request per spec."""
    import torch
    import paper_2206_02362_amd as fw
    from paper_2206_02362_amd.serve import Request
    for k, (nz, nx, vel) in enumerate(mix.pool):
        server.add_model(k, fw.Grid(nz, nx, mix.nb, 2, mix.dx, mix.dx, mix.dt),
                         torch.tensor(vel, dtype=torch.float32, device=dev))
    reqs = []
    for spec in mix.requests:
        x = synth.serve_request_inputs(mix, spec, dev, nt_cap)
        geo = fw.Geometry(x["src_iz"], x["src_ix"], x["rec_iz"], x["rec_ix"], x["wavelet"])
        reqs.append(Request(spec.kind, spec.model, geo, x["nt"], nh=mix.nh, ptilde=x.get("ptilde"),
                            data=x.get("data"), dobs=x.get("dobs"), dso=x.get("dso")))
    return reqs
