#!/usr/bin/env python3
"""Throughput benchmark of the FWIME hot path on one MI355X.

Headline (one "step"): nonlinear modeling of 256 shots on uneven grids --
200 x 600, 300 x 1700 and 500 x 2500 cells at 10 m with a 40-cell absorbing
strip, smooth random 1500-4500 m/s models, Ricker 6-12 Hz, nt 3000-6000,
dt = 0.8 ms, one receiver per column -- as ONE fwime_model_batch call: every
time step of every shot runs in shared two-step stencil launches with an
autotuned tile width.  cell-updates/s counts NZ * NX * (nt - 1) padded
cell-updates per shot.  Inputs are synthetic and seeded and already in HBM.

After the timed steps, each further section runs only while the run stays
inside its wall-clock deadline (a skipped section is recorded as such):
  roofline   the stencil launches of the timed calls (HIP events on the stream
             they run on) against 16 algorithmic bytes per cell-update;
  plain      the same 256 shots one fwime_model call at a time;
  serving    a seeded Poisson request stream (20 requests/s) through the
             request loop and through one-at-a-time FIFO, p50/p99 latency;
  marmousi   one pass of all four operators (modeling, extended Born, its
             adjoint, the gradient) on the 300 x 1700 Marmousi-like set,
             100 shots, nt 5000, 61 offsets;
  time_lag, spline, vp_step   the rows built beyond the hot path;
  cpu_baseline  the FP64 oracle on the host cores (run in worker processes
             beside the GPU sections, never during the timed steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
STENCIL_BYTES = 16         # read u^n, u^{n-1}, V; write u^{n+1}
PROPAGATIONS = {"model": 1, "born_ext_fwd": 2, "born_ext_adj": 2, "gradient": 6}
CSRC = os.path.join(ROOT, "paper_2206_02362_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_multi_batch256_traffic.json")


def log(*a):
    print(f"[{time.perf_counter() - T_START:7.1f} s]", *a, file=sys.stderr, flush=True)


def elapsed() -> float:
    return time.perf_counter() - T_START


# ----------------------------------------------------------------------------
# CPU baseline: the oracle in worker processes (numpy only, one thread each)
# ----------------------------------------------------------------------------

def _cpu_model_task(kind: str, index: int, steps: int):
    """oracle.model on one shot for the first `steps` time steps."""
    import oracle
    import synth
    if kind == "batch":
        w = synth.batch_set(256)[index]
    else:
        w = synth.marmousi_set(100).subset([index])
    steps = min(steps, w.nt)
    g = oracle.Grid(w.nz, w.nx, w.nb, steps, w.dz, w.dx, w.dt, w.sponge_alpha)
    geo = oracle.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix, w.wavelet[:, :steps].copy())
    t = time.perf_counter()
    oracle.model(g, w.vel, geo)
    dt = time.perf_counter() - t
    cells = (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (steps - 1)
    return {"kind": kind, "index": index, "steps": steps, "cells": cells, "s": dt,
            "full_cells": (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1)}


def _cpu_plain_small_task():
    """All four operators of the oracle on the 100 x 200 problem (nt 1500, 11 offsets)."""
    import oracle
    import synth
    w = synth.plain_small()
    g = oracle.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
    geo = oracle.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix, w.wavelet)
    pt = 1e-2 * synth.random_ptilde(w.nh, w.nz, w.nx, 1)
    out = {}
    t = time.perf_counter()
    d = oracle.model(g, w.vel, geo)
    out["model_s"] = time.perf_counter() - t
    t = time.perf_counter()
    oracle.born_ext_fwd(g, w.vel, geo, pt)
    out["born_ext_fwd_s"] = time.perf_counter() - t
    t = time.perf_counter()
    oracle.born_ext_adj(g, w.vel, geo, d, w.nh)
    out["born_ext_adj_s"] = time.perf_counter() - t
    t = time.perf_counter()
    oracle.gradient(g, w.vel, geo, pt, 0.9 * d, 1e-3, synth.dso_weights(w.nh))
    out["gradient_s"] = time.perf_counter() - t
    cells = (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1)
    total = sum(out.values())
    out["cell_updates_per_s"] = sum(PROPAGATIONS.values()) * cells / total
    return out


def _cpu_task(spec):
    if spec[0] == "plain_small":
        return _cpu_plain_small_task()
    return _cpu_model_task(*spec)


def cpu_host():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "model": model}


class CpuBaseline:
    """Starts the oracle runs in a pool of spawned worker processes."""

    def __init__(self, step_cells):
        import multiprocessing as mp
        self.workers = max(2, min(os.cpu_count() or 2, 16) - 2)
        nb = self.workers - 1                      # one worker runs the 100 x 200 four-operator set
        # headline sample: the first nb shots of the 256-shot set, each for
        # about 1.5e8 padded cell-updates (a few hundred time steps)
        self.batch_specs = [("batch", i, max(20, int(1.5e8 / step_cells[i]))) for i in range(nb)]
        # Marmousi-like modeling, shot-parallel: nb shots, 60 steps each
        self.marm_specs = [("marmousi", i, 60) for i in range(nb)]
        specs = [("plain_small",)] + self.batch_specs + self.marm_specs
        saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
        for k in saved:
            os.environ[k] = "1"
        try:
            self.pool = mp.get_context("spawn").Pool(self.workers)
            self.t0 = time.perf_counter()
            self.res = self.pool.map_async(_cpu_task, specs, chunksize=1)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v

    def result(self, timeout: float):
        try:
            out = self.res.get(timeout=max(1.0, timeout))
        except Exception as e:       # timeout or a worker error: report, do not fail the bench
            self.pool.terminate()
            return {"skipped": f"cpu baseline did not finish: {type(e).__name__}"}
        self.pool.close()
        small, rest = out[0], out[1:]
        batch = [r for r in rest if r["kind"] == "batch"]
        marm = [r for r in rest if r["kind"] == "marmousi"]
        # headline sample: shots run concurrently, one per process
        b_cells = sum(r["cells"] for r in batch)
        b_wall = max(r["s"] for r in batch)
        m_rate = sum(r["cells"] / r["s"] for r in marm)
        m_full = 100 * marm[0]["full_cells"]
        return {
            "value": b_cells / b_wall, "unit": "cell-updates/s", "cores": len(batch), "kind": "oracle",
            "sample": f"oracle.model (NumPy FP64, one thread per process) on the first {len(batch)} shots of "
                      f"the 256-shot uneven-grid set, {len(batch)} processes at once, each shot for its first "
                      f"{min(r['steps'] for r in batch)}-{max(r['steps'] for r in batch)} time steps "
                      f"({b_cells:.3g} padded cell-updates in {b_wall:.1f} s); run beside the GPU sections, "
                      f"after the timed steps",
            "host": cpu_host(),
            "plain_100x200_four_ops_one_core": small,
            "marmousi_model_shot_parallel": {
                "processes": len(marm), "steps_per_shot": marm[0]["steps"],
                "cell_updates_per_s": m_rate,
                "extrapolated_100_shots_s": m_full / m_rate,
                "note": "extrapolated from the first 60 steps of one shot per process to 100 shots x 5000 "
                        "steps at the same rate"},
        }


# ----------------------------------------------------------------------------
# GPU sections
# ----------------------------------------------------------------------------

def stencil_source_hash() -> str:
    h = hashlib.sha256()
    for n in ("kernels_step2.hip", "internal.h"):
        h.update(open(os.path.join(CSRC, n), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(launches: int, tile_x: int):
    """HBM bytes per stencil launch of the headline from the committed counter
    runs, or None when those were taken on another kernel version, launch
    count or tile width."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if (rec.get("kernel_source_sha") != stencil_source_hash() or rec.get("launches_per_call") != launches
            or rec.get("tile_x") != tile_x):
        return None
    return rec.get("bytes_per_launch")


def copy_calibration(nbytes: int, reps: int):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty(n, device="cuda:0")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps,
                      "GB_per_s": 2 * n * 4 / dt / 1e9}), flush=True)


def batch_jobs(nshots: int = 256):
    import torch
    import paper_2206_02362_amd as fw
    import synth
    ws = synth.batch_set(nshots)
    vels, jobs, cells = {}, [], []
    for w in ws:
        k = w.extra["size"]
        if k not in vels:
            vels[k] = torch.tensor(w.vel, dtype=torch.float32, device="cuda:0")
        grid = fw.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
        geo = fw.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix,
                          torch.tensor(w.wavelet, dtype=torch.float32, device="cuda:0"))
        data = torch.empty((1, w.nrec, w.nt), device="cuda:0")
        jobs.append((grid, vels[k], geo, data))
        cells.append((w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1))
    return ws, jobs, cells


def plain_compare(ctx, jobs, cells, batched_s):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    for grid, vel, geo, data in jobs:
        ctx.fwime_model(grid, vel, geo, data)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    c = float(sum(cells))
    return {"plain_s": tp, "batched_s": batched_s, "plain_cell_updates_per_s": c / tp,
            "batched_cell_updates_per_s": c / batched_s, "speedup": tp / batched_s,
            "note": "plain = one fwime_model call per shot (one shot per launch, two time steps per launch); "
                    "batched = the headline step (all 256 shots in shared launches)"}


def serve_compare(nreq: int, seed: int = 42, slots: int = 3):
    """The first nreq requests of the seeded Poisson stream (mean 20 requests/s;
    modeling 40 %, extended Born 30 % half forward half adjoint, gradient 30 %;
    grids 200x600 .. 600x3000 at 10 m; 1-32 shots; nt 2000-6000; 11 offsets;
    six resident models), through the request loop (`slots` streams,
    footprint admission, continuous batching of modeling requests) and through
    one-at-a-time FIFO on one context."""
    import torch
    import synth
    import paper_2206_02362_amd as fw
    from paper_2206_02362_amd.serve import Request, Server
    mix = synth.serve_mix(nreq=nreq, seed=seed)

    def requests(srv):
        for k, (nz, nx, v) in enumerate(mix.pool):
            srv.add_model(k, fw.Grid(nz, nx, mix.nb, 2, mix.dx, mix.dx, mix.dt),
                          torch.tensor(v, dtype=torch.float32, device="cuda:0"))
        out = []
        for spec in mix.requests:
            x = synth.serve_request_inputs(mix, spec, "cuda:0")
            geo = fw.Geometry(x["src_iz"], x["src_ix"], x["rec_iz"], x["rec_ix"], x["wavelet"])
            out.append(Request(spec.kind, spec.model, geo, x["nt"], nh=mix.nh, ptilde=x.get("ptilde"),
                               data=x.get("data"), dobs=x.get("dobs"), dso=x.get("dso")))
        return out

    arrivals = [s.arrival for s in mix.requests]
    res = {}
    for name, kw in (("plain_fifo", dict(slots=1, merge_models=1, engine=False)),
                     ("served", dict(slots=slots, engine=True, policy="fcfs")),
                     ("served_short_first", dict(slots=slots, engine=True, policy="short_first"))):
        srv = Server(0, **kw)
        reqs = requests(srv)
        torch.cuda.synchronize()
        log(f"serve replay ({name}): {len(reqs)} requests")
        done = srv.replay(reqs, arrivals)
        torch.cuda.synchronize()
        errs = [r for r in done if r.error is not None]
        if errs:
            raise RuntimeError(f"{len(errs)} requests failed, first: {errs[0].error}")
        st = Server.stats(done)
        st["peak_reserved_bytes"] = srv.peak_reserved
        st["budget_bytes"] = srv.budget
        res[name] = st
        log(f"  {name}: p50 {st['p50_s']:.2f} s, p99 {st['p99_s']:.2f} s, makespan {st['makespan_s']:.2f} s")
        srv.close()
        del srv, reqs, done
        torch.cuda.empty_cache()
    kinds = {}
    for s_ in mix.requests:
        kinds[s_.kind] = kinds.get(s_.kind, 0) + 1
    return {"workload": f"first {nreq} requests of a Poisson stream at 20/s (seed {seed}), kinds {kinds}, grids "
                        f"200x600..600x3000, 1-32 shots, nt 2000-6000, nh {mix.nh}, {len(mix.pool)} resident models",
            "arrival_span_s": arrivals[-1], "samples": nreq, "slots": slots, **res,
            "ratios_over_plain_fifo": {
                k: {"throughput": res[k]["cell_updates_per_s"] / res["plain_fifo"]["cell_updates_per_s"],
                    "p50": res[k]["p50_s"] / res["plain_fifo"]["p50_s"],
                    "p99": res[k]["p99_s"] / res["plain_fifo"]["p99_s"]}
                for k in ("served", "served_short_first")},
            "note": "plain_fifo: one request at a time on one stream; served: 3 slot streams for extended-Born and "
                    "gradient requests plus the continuous-batching engine for modeling requests, admission in "
                    "arrival order by HBM footprint and by stencil workgroups (beside running requests a request "
                    "starts only while all their workgroups per launch stay within 4096, so requests that fill "
                    "the GPU run alone and small ones overlap); served_short_first: the same with the least-work "
                    "request that can start first (aging bound 30 s). With fewer than 100 samples p99 is close "
                    "to the maximum latency"}


def serve_estimate_s(nreq: int, rate: float = 1.5e11) -> float:
    """Rough GPU seconds of the served + FIFO replays of the first nreq requests."""
    import synth
    from paper_2206_02362_amd.serve import PROPAGATIONS as SP
    mix = synth.serve_mix(nreq=nreq, seed=42, velocities=False)
    cells = 0.0
    for s in mix.requests:
        nz, nx, _ = mix.pool[s.model]
        extra = {"model": 1.0, "born_fwd": 1.0, "born_adj": 1.5, "gradient": 1.4}[s.kind]
        cells += extra * SP[s.kind] * len(s.src_ix) * (nz + 2 * mix.nb) * (nx + 2 * mix.nb) * (s.nt - 1)
    return 3.0 * cells / rate + 8.0


def marmousi_pass(ctx, nt: int = 0):
    import torch
    import paper_2206_02362_amd as fw
    import synth
    w = synth.marmousi_set(100)
    if nt > 0:                       # counter runs: a shorter time axis, the same launch shapes
        w.nt = min(nt, w.nt)
        w.wavelet = w.wavelet[:, :w.nt].copy()
    dev = "cuda:0"
    grid = fw.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
    vel = torch.tensor(w.vel, dtype=torch.float32, device=dev)
    geo = fw.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix, torch.tensor(w.wavelet, dtype=torch.float32, device=dev))
    vtrue = torch.tensor(w.vel * (1.0 + 0.03 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 77, 300.0)),
                         dtype=torch.float32, device=dev)
    ptilde = torch.tensor(1e-2 * synth.random_ptilde(w.nh, w.nz, w.nx, 78), dtype=torch.float32, device=dev)
    dso = synth.dso_weights(w.nh)
    dobs = ctx.model(grid, vtrue, geo)
    torch.cuda.synchronize()
    times = {}
    for name, call in (("model", lambda: ctx.model(grid, vel, geo)),
                       ("born_ext_fwd", lambda: ctx.born_ext_fwd(grid, vel, geo, ptilde)),
                       ("born_ext_adj", lambda: ctx.born_ext_adj(grid, vel, geo, dobs, w.nh)),
                       ("gradient", lambda: ctx.gradient(grid, vel, geo, ptilde, dobs, 1e-4, dso))):
        t = time.perf_counter()
        out = call()
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t
        del out
    per_prop = w.nshots * (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1)
    total = sum(times.values())
    # modeling with a free surface at the top of the model (the paper's
    # Marmousi2 variant with free-surface multiples), same shots
    gfs = fw.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha, True)
    t = time.perf_counter()
    out = ctx.model(gfs, vel, geo)
    torch.cuda.synchronize()
    t_fs = time.perf_counter() - t
    del out
    return {"workload": f"{w.name}: {w.nshots} shots, nt {w.nt}, nh {w.nh}, padded "
                        f"{w.nz + 2 * w.nb}x{w.nx + 2 * w.nb}, one pass of each operator (first calls)",
            "seconds": times, "total_s": total, "model_free_surface_s": t_fs,
            "cell_updates_per_s": sum(PROPAGATIONS.values()) * per_prop / total,
            "note": "propagations counted as in the paper's cost analysis: modeling 1, extended Born 2, "
                    "adjoint 2, gradient 6 per shot; checkpoint recomputations not counted"}, (grid, vel, geo, dobs, w)


def time_lag_section(ctx, grid, vel, geo, w, nshots=8):
    import torch
    import paper_2206_02362_amd as fw
    import synth
    ctx.trim()
    torch.cuda.empty_cache()
    ns = min(nshots, w.nshots)
    ntau, lag = 101, max(1, int(round(0.016 / w.dt)))
    gsub = fw.Geometry(w.src_iz[:ns], w.src_ix[:ns], w.rec_iz[:ns], w.rec_ix[:ns], geo.wavelet[:ns].contiguous())
    ptau = torch.tensor(1e-2 * synth.random_ptilde(ntau, w.nz, w.nx, 79), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    t = time.perf_counter()
    dtau = ctx.born_ext_tau_fwd(grid, vel, gsub, ptau, lag)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t
    t = time.perf_counter()
    dtau = ctx.born_ext_tau_fwd(grid, vel, gsub, ptau, lag)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t
    t = time.perf_counter()
    ctx.born_ext_tau_adj(grid, vel, gsub, dtau, ntau, lag)
    torch.cuda.synchronize()
    t_a = time.perf_counter() - t
    # the time-lag FWIME gradient on the same shots (objective, both
    # gradients; first call); a failure is recorded, not raised
    t_g, g_err = None, None
    try:
        dobs_sub = (dtau * 1.01).contiguous()
        dso = synth.dso_weights(ntau)
        t = time.perf_counter()
        ctx.gradient_tau(grid, vel, gsub, ptau, lag, dobs_sub, 1e-4, dso)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t
    except Exception as e:              # reported in the record
        g_err = f"{type(e).__name__}: {e}"
    cells = ns * (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1)
    return {"workload": f"{w.name}: {ns} shots, nt {w.nt}, ntau {ntau}, lag {lag} steps ({lag * w.dt * 1e3:.0f} ms)",
            "fwd_s": t_f, "adj_s": t_a, "gradient_s": t_g, "gradient_error": g_err, "fwd_first_call_s": t_cold,
            "fwd_cell_updates_per_s": 2 * cells / t_f, "adj_cell_updates_per_s": 2 * cells / t_a,
            "lag_terms_per_s_fwd": ntau * ns * w.nz * w.nx * (w.nt - 1) / t_f}


def spline_section(ctx, w, reps=50):
    import numpy as np
    import torch
    import synth
    zn = np.unique(np.concatenate([np.arange(0, w.nz - 1, 10), [w.nz - 1],
                                   np.arange(w.nz // 3 - 20, w.nz // 3 + 20, 5)]) * w.dz)
    xn = np.unique(np.concatenate([np.arange(0, w.nx - 1, 10), [w.nx - 1]]) * w.dx)
    mc = torch.tensor(synth.gaussian_perturbation(len(zn), len(xn), w.dx, 80, 30.0), dtype=torch.float32,
                      device="cuda:0")
    fine = torch.empty((w.nx, w.nz), dtype=torch.float32, device="cuda:0")
    back = torch.empty((len(xn), len(zn)), dtype=torch.float32, device="cuda:0")
    times = {}
    for name, call in (("apply", lambda: ctx.fwime_spline_apply(w.nz, w.nx, w.dz, w.dx, zn, xn, mc, fine)),
                       ("adjoint", lambda: ctx.fwime_spline_adjoint(w.nz, w.nx, w.dz, w.dx, zn, xn, fine, back))):
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) * 1e3 / reps
    return {"workload": f"{w.nz}x{w.nx} model grid, {len(zn)}x{len(xn)} spline nodes",
            "apply_us_per_call": times["apply"], "adjoint_us_per_call": times["adjoint"]}


def vp_section(ctx, grid, vel, geo, dobs, w, iters=2):
    import torch
    import synth
    dso = synth.dso_weights(w.nh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.vp_solve(grid, vel, geo, dobs, w.nh, 0.0, dso, 0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    _, phi = ctx.vp_solve(grid, vel, geo, dobs, w.nh, 0.0, dso, iters)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t
    per_iter = (t_all - t_setup) / iters
    per_prop = w.nshots * (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1)
    return {"iterations": iters, "s_setup": t_setup, "s_per_iteration": per_iter,
            "cell_updates_per_s": 4 * per_prop / per_iter, "objective": [float(x) for x in phi]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--deadline-s", type=float, default=480.0,
                    help="wall-clock budget from process start; optional sections past it are skipped")
    ap.add_argument("--sections", default="roofline,plain,cpu,serving,marmousi,time_lag,spline,vp",
                    help="comma list of the sections to run after the timed steps")
    ap.add_argument("--serve-requests", type=int, default=0, help="requests in the serving replay (0: fit)")
    ap.add_argument("--marmousi-nt", type=int, default=0,
                    help="time steps of the four-operator section (0: the workload's 5000); for counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(shots would shard across GPUs with one all-reduce of the gradients).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2206_02362_amd as fw

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.copy_calibration:
        copy_calibration(1 << 30, 5)
        return
    sections = set(s for s in args.sections.split(",") if s)
    deadline = args.deadline_s

    def fits(name, est):
        if name not in sections:
            return False
        left = deadline - elapsed()
        if est > left:
            log(f"section {name} skipped: needs about {est:.0f} s, {left:.0f} s left")
            skipped[name] = {"skipped": "deadline", "estimate_s": est, "left_s": left}
            return False
        return True

    skipped = {}
    ws, jobs, cells = batch_jobs(256)
    total_cells = float(sum(cells))
    log(f"headline: {len(jobs)} shots on 200x600 / 300x1700 / 500x2500, {total_cells:.4g} cell-updates per step")
    ctx = fw.Context(0)
    ctx.set_timing(True)
    for i in range(args.warmup):
        t = time.perf_counter()
        ctx.fwime_model_batch(jobs)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t:.2f} s (tile width {ctx.info()['last_batch_tile_x']})")
    launches, kern_ms = 0, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.fwime_model_batch(jobs)
        inf = ctx.info()                 # waits for the call's last stencil launch
        launches += inf["last_stencil_launches"]
        kern_ms += inf["last_stencil_ms"]
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = 1e3 * t_steps / args.steps
    value = total_cells / (t_steps / args.steps)
    log(f"timed: {args.steps} steps, {ms_per_step:.1f} ms per step, {value:.4g} cell-updates/s")

    # roofline of the dominant kernel (k_step2_multi): algorithmic bytes of the
    # timed calls over the event time of their stencil launches
    algo_bytes = STENCIL_BYTES * total_cells * args.steps
    per_launch_us = 1e3 * kern_ms / launches
    achieved = algo_bytes / (kern_ms / 1e3)
    lpc = launches // args.steps
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": achieved / PEAK_HBM, "traffic": measured_traffic(lpc, ctx.info()["last_batch_tile_x"]),
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": f"k_step2_multi<{ctx.info()['last_batch_tile_x']}> (two stencil time steps per launch, "
                          f"all active shots of all grids)",
                "launches_per_call": lpc, "avg_launch_us": per_launch_us,
                "bytes_per_launch": algo_bytes / launches,
                "stencil_share_of_step": kern_ms / (1e3 * t_steps)}
    log(f"stencil: {per_launch_us:.1f} us per launch, {achieved / 1e9:.0f} GB/s algorithmic "
        f"({roofline['frac']:.3f} of 8 TB/s)")

    plain = serving = marm = tau = spline = vp = None
    cpu = None
    if fits("plain", 2.6 * t_steps / args.steps + 5):
        plain = plain_compare(ctx, jobs, cells, t_steps / args.steps)
        log(f"plain: {plain['plain_s']:.2f} s, batched {plain['speedup']:.2f}x faster")
    del jobs
    ctx.trim()
    torch.cuda.empty_cache()

    cpu_job = None
    if "cpu" in sections and deadline - elapsed() > 60:
        cpu_job = CpuBaseline([(w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) for w in ws])
        log(f"cpu baseline started in {cpu_job.workers} worker processes")

    if "serving" in sections:
        n = args.serve_requests
        if n <= 0:
            n = 0
            for cand in (96, 80, 64, 48, 40, 32, 24, 16):
                if serve_estimate_s(cand) < 0.6 * (deadline - elapsed() - 30):
                    n = cand
                    break
        if n and fits("serving", serve_estimate_s(n)):
            serving = serve_compare(n)
        elif not n:
            skipped["serving"] = {"skipped": "deadline"}

    marm_ctx = None
    if fits("marmousi", 47):
        marm, marm_ctx = marmousi_pass(ctx, args.marmousi_nt)
        log(f"marmousi four-operator pass: {marm['total_s']:.1f} s")
    if marm_ctx is not None:
        grid, vel, geo, dobs, w = marm_ctx
        if fits("time_lag", 25):
            tau = time_lag_section(ctx, grid, vel, geo, w)
            log(f"time lag: forward {tau['fwd_s']:.2f} s, adjoint {tau['adj_s']:.2f} s, gradient "
                + (f"{tau['gradient_s']:.2f} s" if tau["gradient_s"] is not None else tau["gradient_error"]))
        if fits("spline", 3):
            spline = spline_section(ctx, w)
        if fits("vp", 45):
            ctx.trim()
            torch.cuda.empty_cache()
            vp = vp_section(ctx, grid, vel, geo, dobs, w)
            log(f"vp: {vp['s_per_iteration']:.2f} s per CG iteration")
        del marm_ctx, grid, vel, geo, dobs

    if cpu_job is not None:
        cpu = cpu_job.result(deadline + 60 - elapsed())
        log(f"cpu baseline: {cpu.get('value', 0):.4g} cell-updates/s")
    elif "cpu" in sections:
        cpu = {"skipped": "deadline"}

    rec = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch-256: 256 modeling shots on uneven grids (200x600, 300x1700, 500x2500 at "
                               "10 m, 40-cell strip), nt 3000-6000, Ricker 6-12 Hz, one fwime_model_batch call "
                               "per step",
                   "nshots": 256, "cell_updates_per_step": total_cells},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_vs_plain": plain,
        "serving": serving,
        "marmousi_four_ops": marm,
        "time_lag": tau,
        "spline": spline,
        "vp_step": vp,
        "skipped": skipped or None,
        "wall_s": elapsed(),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
