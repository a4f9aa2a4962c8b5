#!/usr/bin/env python3
"""Throughput benchmark of the FWIME hot path on one MI355X.

One step = one pass of every operator of the hot path over the whole shot set:
nonlinear modeling f(m), extended Born B~(m) p~, its adjoint B~^T d and the
FWIME objective with both gradients, each through the C ABI.  The workload is
the Marmousi-like 300 x 1700 grid (10 m, 60-cell absorbing strip, padded
420 x 1820), 100 shots every 170 m, 1700 receivers, 8 Hz Ricker, dt = 0.8 ms,
nt = 5000, 61 subsurface offsets; inputs are synthetic and seeded.

cell-updates/s counts propagations as the paper's cost analysis does
(Section "Computational aspects": modeling 1, extended Born 2, its adjoint 2,
gradient 6 per shot), each NZ * NX * (nt - 1) padded cell-updates; recomputed
propagations of the checkpointing scheme are not counted.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
STENCIL_BYTES = 16         # read u^n, u^{n-1}, V; write u^{n+1}
PROPAGATIONS = {"model": 1, "born_ext_fwd": 2, "born_ext_adj": 2, "gradient": 6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


CSRC = os.path.join(ROOT, "paper_2206_02362_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_traffic.json")


def two_step() -> bool:
    """The library runs two time steps per stencil launch unless FWIME_STEP1 is set."""
    v = os.environ.get("FWIME_STEP1")
    return not (v and int(v) != 0)


def stencil_source_hash() -> str:
    """Hash of the sources that define the dominant stencil kernel."""
    names = ["kernels_step2.hip", "internal.h"] if two_step() else ["kernels_step.hip", "internal.h"]
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(CSRC, n), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(nshots: int, nt: int):
    """HBM bytes per stencil launch from the committed counter runs, or None
    when those counters were taken on another version of the kernel or
    another launch shape."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != stencil_source_hash() or rec.get("shots_per_launch") != nshots:
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


def make_workload(name: str, nshots: int | None):
    import synth
    if name == "marmousi":
        w = synth.marmousi_set(100 if nshots is None else nshots)
    elif name == "plain-small":
        w = synth.plain_small()
    else:
        raise SystemExit(f"unknown workload {name}")
    return w


def cpu_baseline(w, steps: int):
    """The FP64 oracle on a bounded sample: one shot, the first `steps` time steps."""
    import numpy as np
    import oracle
    import synth
    sub = w.subset([0])
    g = oracle.Grid(sub.nz, sub.nx, sub.nb, steps, sub.dz, sub.dx, sub.dt, sub.sponge_alpha)
    geo = oracle.Geometry(sub.src_iz, sub.src_ix, sub.rec_iz, sub.rec_ix, sub.wavelet[:, :steps].copy())
    t = time.perf_counter()
    oracle.model(g, sub.vel, geo)
    dt = time.perf_counter() - t
    cells = (sub.nz + 2 * sub.nb) * (sub.nx + 2 * sub.nb) * (steps - 1)
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle.model, 1 shot of the {sub.nz}x{sub.nx} workload, first {steps} time steps "
                      f"({cells:.3g} padded cell-updates in {dt:.1f} s, NumPy FP64, one thread)"}


def batch_compare(ctx, nshots: int = 256):
    """256 shots on three grid sizes (200x600, 300x1700, 500x2500), nt 3000-6000:
    one fwime_model_batch call (all shots per launch, graph-replayed, autotuned
    tile width) against the plain path, one fwime_model call per shot."""
    import torch
    import paper_2206_02362_amd as fw
    import synth
    ws = synth.batch_set(nshots)
    vels = {}
    jobs = []
    cells = 0
    for w in ws:
        k = w.extra["size"]
        if k not in vels:
            vels[k] = torch.tensor(w.vel, dtype=torch.float32, device="cuda:0")
        grid = fw.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
        geo = fw.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix,
                          torch.tensor(w.wavelet, dtype=torch.float32, device="cuda:0"))
        data = torch.empty((1, w.nrec, w.nt), device="cuda:0")
        jobs.append((grid, vels[k], geo, data))
        cells += (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (w.nt - 1)
    log(f"batch compare: {len(jobs)} jobs, {cells:.3g} cell-updates")
    ctx.fwime_model_batch(jobs)          # first call tunes the tile width
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.fwime_model_batch(jobs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    log(f"batched: {tb:.2f} s")
    t = time.perf_counter()
    for grid, vel, geo, data in jobs:
        ctx.fwime_model(grid, vel, geo, data)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    log(f"plain: {tp:.2f} s")
    return {"workload": f"{len(jobs)} shots on 200x600 / 300x1700 / 500x2500 grids (40-cell strip), "
                        f"nt 3000-6000, Ricker 6-12 Hz, modeling",
            "cell_updates": cells, "batched_s": tb, "plain_s": tp,
            "batched_cell_updates_per_s": cells / tb, "plain_cell_updates_per_s": cells / tp,
            "speedup": tp / tb, "tile_x": ctx.info()["last_batch_tile_x"]}


def serve_compare(nreq: int, seed: int = 42, slots: int = 3):
    """A seeded Poisson stream (mean 20 requests/s) of modeling 40 %, extended
    Born 30 % (half forward, half adjoint) and gradient 30 % requests on grids
    from 200x600 to 600x3000 (10 m, 40-cell strip), 1-32 shots, nt 2000-6000,
    11 offsets, over six resident models: the request loop (`slots` streams,
    footprint admission, merged modeling) against plain first-come-first-served
    (one request at a time, one context, no merging)."""
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
    for name, kw in (("plain_fifo", dict(slots=1, merge_models=1)), ("served", dict(slots=slots, merge_models=8))):
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
        for s_ in srv.slots:
            s_.ctx.close()
        del srv, reqs, done
        torch.cuda.empty_cache()
    kinds = {}
    for s_ in mix.requests:
        kinds[s_.kind] = kinds.get(s_.kind, 0) + 1
    return {"workload": f"{nreq} requests, Poisson 20/s (seed {seed}), kinds {kinds}, grids 200x600..600x3000, "
                        f"1-32 shots, nt 2000-6000, nh {mix.nh}, {len(mix.pool)} resident models",
            "slots": slots, **res,
            "throughput_speedup": res["served"]["cell_updates_per_s"] / res["plain_fifo"]["cell_updates_per_s"],
            "p99_ratio_served_over_plain": res["served"]["p99_s"] / res["plain_fifo"]["p99_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="marmousi")
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--ops", default="model,born_ext_fwd,born_ext_adj,gradient")
    ap.add_argument("--cpu-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nt", type=int, default=None, help="shorten the time axis (counter runs)")
    ap.add_argument("--no-batch-compare", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=16, help="requests in the serving replay (0: skip)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving replay")
    ap.add_argument("--vp-iters", type=int, default=2,
                    help="CG iterations of the variable-projection step to time (0: skip)")
    ap.add_argument("--tau-shots", type=int, default=8,
                    help="shots of the time-lag extended Born pair to time (0: skip)")
    ap.add_argument("--spline-reps", type=int, default=50,
                    help="calls of the spline operator S and its adjoint to time (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(shots would shard across GPUs with one all-reduce of the gradients).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2206_02362_amd as fw
    import synth

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.copy_calibration:
        copy_calibration(1 << 30, 5)
        return
    if args.serve_only:
        print(json.dumps({"serving": serve_compare(args.serve_requests)}), flush=True)
        return
    ops = [o for o in args.ops.split(",") if o]
    w = make_workload(args.workload, args.shots)
    if args.nt is not None:
        w.nt = args.nt
        w.wavelet = w.wavelet[:, :args.nt].copy()
    log(f"workload {w.name}: {w.nshots} shots, nt {w.nt}, nh {w.nh}, padded {w.nz + 2 * w.nb}x{w.nx + 2 * w.nb}")
    dev = "cuda:0"
    ctx = fw.Context(0)
    grid = fw.Grid(w.nz, w.nx, w.nb, w.nt, w.dz, w.dx, w.dt, w.sponge_alpha)
    vel = torch.tensor(w.vel, dtype=torch.float32, device=dev)
    geo = fw.Geometry(w.src_iz, w.src_ix, w.rec_iz, w.rec_ix,
                      torch.tensor(w.wavelet, dtype=torch.float32, device=dev))
    vtrue = torch.tensor(w.vel * (1.0 + 0.03 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 77, 300.0)),
                         dtype=torch.float32, device=dev)
    ptilde = torch.tensor(1e-2 * synth.random_ptilde(w.nh, w.nz, w.nx, 78), dtype=torch.float32, device=dev)
    dso = synth.dso_weights(w.nh)
    log("setup: observed data")
    dobs = ctx.model(grid, vtrue, geo)
    torch.cuda.synchronize()

    outs = {}

    def step():
        if "model" in ops:
            outs["model"] = ctx.model(grid, vel, geo)
        if "born_ext_fwd" in ops:
            outs["born"] = ctx.born_ext_fwd(grid, vel, geo, ptilde)
        if "born_ext_adj" in ops:
            outs["adj"] = ctx.born_ext_adj(grid, vel, geo, dobs, w.nh)
        if "gradient" in ops:
            outs["grad"] = ctx.gradient(grid, vel, geo, ptilde, dobs, 1e-4, dso)

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t:.2f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    NZ, NX = w.nz + 2 * w.nb, w.nx + 2 * w.nb
    per_prop = w.nshots * NZ * NX * (w.nt - 1)
    nprop = sum(PROPAGATIONS[o] for o in ops)
    value = nprop * per_prop / (elapsed / args.steps)

    # Dominant kernel: the stencil.  fwime_model is ceil((nt - 1) / 2) launches
    # of the two-step kernel (nt - 1 of the one-step kernel with FWIME_STEP1=1),
    # all shots in one launch, plus one receiver gather; time it with events on
    # the stream the library launches on.
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    data = torch.empty((w.nshots, w.nrec, w.nt), device=dev)
    ctx.fwime_model(grid, vel, geo, data)      # tables and arena warm
    torch.cuda.synchronize()
    reps = 2
    tev = 0.0
    for _ in range(reps):
        # the bracket also holds the call's validation reduction and table upload
        e0.record(st)
        ctx.fwime_model(grid, vel, geo, data)
        e1.record(st)
        e1.synchronize()
        tev += e0.elapsed_time(e1) / 1e3
    steps_per_launch = 2 if two_step() else 1
    launches = (w.nt - 1 + steps_per_launch - 1) // steps_per_launch
    per_launch = tev / reps / launches
    step_bytes = STENCIL_BYTES * w.nshots * NZ * NX          # algorithmic bytes of one time step
    achieved = step_bytes * (w.nt - 1) / (tev / reps)
    kname = ("k_step2 (two stencil time steps per launch, all shots)" if steps_per_launch == 2
             else "k_step (one stencil time step per launch, all shots)")
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": achieved / PEAK_HBM, "traffic": measured_traffic(w.nshots, w.nt),
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": kname, "steps_per_launch": steps_per_launch,
                "bytes_per_launch": step_bytes * steps_per_launch, "avg_launch_us": per_launch * 1e6}
    log(f"stencil: {per_launch * 1e6:.1f} us per launch ({steps_per_launch} steps), "
        f"{achieved / 1e9:.0f} GB/s algorithmic")

    batch = None
    if not args.no_batch_compare:
        batch = batch_compare(ctx)

    vp = None
    if args.vp_iters > 0:
        # variable-projection step (eq. vp.obj): model + B~* once, then B~ and
        # B~* per CG iteration; timed as a whole and per iteration
        outs.clear()
        log(f"variable-projection step: {args.vp_iters} CG iterations")
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, phi = ctx.vp_solve(grid, vel, geo, dobs, w.nh, 0.0, dso, 0)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t
        t = time.perf_counter()
        _, phi = ctx.vp_solve(grid, vel, geo, dobs, w.nh, 0.0, dso, args.vp_iters)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t
        per_iter = (t_all - t_setup) / args.vp_iters
        vp = {"iterations": args.vp_iters, "eps": 0.0, "s_total": t_all, "s_setup": t_setup,
              "s_per_iteration": per_iter,
              "cell_updates_per_s": 4 * per_prop / per_iter,
              "note": "setup = f(m) and B~* once (3 propagations/shot); each CG iteration = B~ + B~* "
                      "(4 propagations/shot counted)",
              "objective": [float(x) for x in phi]}
        log(f"vp: {per_iter:.2f} s per CG iteration, objective {vp['objective']}")

    tau = None
    if args.tau_shots > 0 and max(1, int(round(0.016 / w.dt))) * 100 > 4 * w.nt:
        log("time-lag extension skipped: the record is too short for 101 lags of 16 ms")
    elif args.tau_shots > 0:
        # extended Born with time lags: 101 lags of 16 ms (the paper's Marmousi2
        # setting) on the first shots of the workload; each shot's background
        # history is about 2 nt padded fields, so only a few shots fit at once;
        # the context's arena and solver buffers are released first, or the
        # batches shrink to a shot or two
        outs.clear()
        ctx.trim()
        torch.cuda.empty_cache()
        ns_tau = min(args.tau_shots, w.nshots)
        ntau, lag = 101, max(1, int(round(0.016 / w.dt)))
        gsub = fw.Geometry(w.src_iz[:ns_tau], w.src_ix[:ns_tau], w.rec_iz[:ns_tau], w.rec_ix[:ns_tau],
                           geo.wavelet[:ns_tau].contiguous())
        ptau = torch.tensor(1e-2 * synth.random_ptilde(ntau, w.nz, w.nx, 79), dtype=torch.float32, device=dev)
        log(f"time-lag extension: {ns_tau} shots, ntau {ntau}, lag {lag} steps")
        # one untimed call grows the context's arena to the histories' size
        # (after the larger earlier sections that first allocation alone takes
        # seconds), as the other sections time warm calls
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
        img = ctx.born_ext_tau_adj(grid, vel, gsub, dtau, ntau, lag)
        torch.cuda.synchronize()
        t_a = time.perf_counter() - t
        cells = ns_tau * NZ * NX * (w.nt - 1)
        tau = {"workload": f"{w.name}: {ns_tau} shots, nt {w.nt}, ntau {ntau}, lag {lag} steps "
                           f"({lag * w.dt * 1e3:.0f} ms)",
               "fwd_s": t_f, "adj_s": t_a, "fwd_first_call_s": t_cold,
               "fwd_cell_updates_per_s": 2 * cells / t_f, "adj_cell_updates_per_s": 2 * cells / t_a,
               "lag_terms_per_s_fwd": ntau * ns_tau * w.nz * w.nx * (w.nt - 1) / t_f,
               "note": "two propagations per shot counted per operator; lag terms = ntau multiply-adds "
                       "per model cell and step"}
        log(f"time lag: forward {t_f:.2f} s (first call {t_cold:.2f} s), adjoint {t_a:.2f} s")
        del dtau, img, ptau

    spline = None
    if args.spline_reps > 0:
        # S and S* on the model grid, nodes every 10 cells plus a refined band
        # of 5-cell spacing around an interface at a third of the depth
        zn = np.unique(np.concatenate([np.arange(0, w.nz - 1, 10), [w.nz - 1],
                                       np.arange(w.nz // 3 - 20, w.nz // 3 + 20, 5)]) * w.dz)
        xn = np.unique(np.concatenate([np.arange(0, w.nx - 1, 10), [w.nx - 1]]) * w.dx)
        mc = torch.tensor(synth.gaussian_perturbation(len(zn), len(xn), w.dx, 80, 30.0), dtype=torch.float32,
                          device=dev)
        fine = torch.empty((w.nx, w.nz), dtype=torch.float32, device=dev)
        back = torch.empty((len(xn), len(zn)), dtype=torch.float32, device=dev)
        times = {}
        for name, call in (("apply", lambda: ctx.fwime_spline_apply(w.nz, w.nx, w.dz, w.dx, zn, xn, mc, fine)),
                           ("adjoint", lambda: ctx.fwime_spline_adjoint(w.nz, w.nx, w.dz, w.dx, zn, xn, fine,
                                                                        back))):
            call()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.spline_reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) * 1e3 / args.spline_reps
        spline = {"workload": f"{w.nz}x{w.nx} model grid, {len(zn)}x{len(xn)} spline nodes",
                  "apply_us_per_call": times["apply"], "adjoint_us_per_call": times["adjoint"],
                  "note": "whole calls (node upload with one stream synchronization, axis tables, "
                          "interpolation); per-kernel times in the rocprofv3 summary"}
        log(f"spline: apply {times['apply']:.1f} us, adjoint {times['adjoint']:.1f} us per call")
        del fine, back, mc

    serving = None
    if args.serve_requests > 0:
        # give the device memory of the step back to the server's budget
        outs.clear()
        del data
        ctx.trim()
        torch.cuda.empty_cache()
        serving = serve_compare(args.serve_requests)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps")
        cpu = cpu_baseline(w, args.cpu_steps)

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
        "config": {"workload": f"{w.name}: {w.nshots} shots, nt {w.nt}, nh {w.nh}, padded {NZ}x{NX}, "
                               f"ops {'+'.join(ops)} ({nprop} propagations/shot counted)",
                   "nshots": w.nshots, "nt": w.nt, "nh": w.nh, "padded_cells": NZ * NX,
                   "model_cells": w.nz * w.nx},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_vs_plain": batch,
        "vp_step": vp,
        "time_lag": tau,
        "spline": spline,
        "serving": serving,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
