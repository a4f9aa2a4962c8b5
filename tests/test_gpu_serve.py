"""Request loop on the GPU: each result is the same alone and in the mix.

A seeded Poisson stream of modeling, extended Born (forward and adjoint) and
gradient requests runs through the server (several slots, overlapping
streams, merged modeling requests, admission by HBM footprint).  Each
request is then run alone, one at a time, on a fresh context.  Modeling
results must agree bit for bit (the per-cell arithmetic does not depend on
the launch); the others to relative L2 <= 1e-6 (only the order of the
per-shot sums may differ, when free memory splits the shots differently).
Every served result of a small mix is also compared with the FP64 oracle
(relative L2 <= 1e-4).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from _helpers import rel_l2, serve_setup

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _alone(reqs, server):
    import torch
    import paper_2206_02362_amd as fw
    ctx = fw.Context(0)
    out = []
    for r in reqs:
        grid = server.grid_for(r)
        _, vel = server.models[r.model]
        if r.kind == "model":
            out.append(ctx.model(grid, vel, r.geom))
        elif r.kind == "born_fwd":
            out.append(ctx.born_ext_fwd(grid, vel, r.geom, r.ptilde))
        elif r.kind == "born_adj":
            out.append(ctx.born_ext_adj(grid, vel, r.geom, r.data, r.nh))
        else:
            out.append(ctx.gradient(grid, vel, r.geom, r.ptilde, r.dobs, r.eps, r.dso))
        torch.cuda.synchronize()
    ctx.close()
    return out


def _compare(reqs, alone):
    worst = 0.0
    for r, a in zip(reqs, alone):
        assert r.error is None, (r.id, r.kind, r.error)
        if r.kind == "model":
            assert np.array_equal(r.result.cpu().numpy(), a.cpu().numpy()), (r.id, r.merged)
        elif r.kind in ("born_fwd", "born_adj"):
            e = rel_l2(r.result.cpu().numpy(), a.cpu().numpy())
            worst = max(worst, e)
            assert e <= 1e-6, (r.id, r.kind, e)
        else:
            for x, y in zip(r.result, a):
                e = rel_l2(x.cpu().numpy(), y.cpu().numpy())
                worst = max(worst, e)
                assert e <= 1e-6, (r.id, r.kind, e)
    return worst


def _small_mix(seed):
    return synth.serve_mix(nreq=14, seed=seed, rate=400.0, npool=3, nz_choices=(30, 40, 50),
                           nx_choices=(50, 70, 90), shots=(1, 4), nt_choices=(150, 200, 260), dt=1e-3,
                           nb=8, nh=5)


@pytest.mark.parametrize("engine", [True, False])
def test_serve_mix_equals_alone(engine):
    import torch
    from paper_2206_02362_amd.serve import Server
    say(f"case: 14-request mix, 3 slots, {'continuous batching engine' if engine else 'merging at admission'}")
    mix = _small_mix(5)
    srv = Server(0, slots=3, engine=engine, engine_steps=16)
    reqs = serve_setup(mix, srv)
    torch.cuda.synchronize()
    srv.replay(reqs, [s.arrival for s in mix.requests])
    torch.cuda.synchronize()
    assert srv.reserved == 0 and srv.peak_reserved <= srv.budget
    assert sorted(srv.admit_order) == srv.admit_order
    say("  merged groups:", sorted({r.merged for r in reqs}), "kinds:", [r.kind for r in reqs])
    worst = _compare(reqs, _alone(reqs, srv))
    say("  worst rel L2 (non-modeling):", worst)
    srv.close()


def _oracle_result(r, server):
    """The FP64 oracle's result for a served request (float32 inputs as float64)."""
    grid = server.grid_for(r)
    gm, vel = server.models[r.model]
    g = oracle.Grid(grid.nz, grid.nx, grid.nb, grid.nt, grid.dz, grid.dx, grid.dt, grid.sponge_alpha)
    h = lambda t: t.detach().double().cpu().numpy()
    geo = oracle.Geometry(r.geom.src_iz, r.geom.src_ix, r.geom.rec_iz, r.geom.rec_ix, h(r.geom.wavelet))
    v = h(vel)
    if r.kind == "model":
        return oracle.model(g, v, geo)
    if r.kind == "born_fwd":
        return oracle.born_ext_fwd(g, v, geo, h(r.ptilde))
    if r.kind == "born_adj":
        return oracle.born_ext_adj(g, v, geo, h(r.data), r.nh)
    return oracle.gradient(g, v, geo, h(r.ptilde), h(r.dobs), r.eps, r.dso)


def test_serve_mix_matches_oracle():
    import torch
    from paper_2206_02362_amd.serve import Server
    say("case: 14-request mix, 3 slots and the engine, every result vs the oracle")
    mix = _small_mix(5)
    srv = Server(0, slots=3, engine=True, engine_steps=16)
    reqs = serve_setup(mix, srv)
    torch.cuda.synchronize()
    srv.replay(reqs, [s.arrival for s in mix.requests])
    torch.cuda.synchronize()
    for r in reqs:
        assert r.error is None, (r.id, r.kind, r.error)
        ref = _oracle_result(r, srv)
        if r.kind == "gradient":
            obj, gv, gp = r.result
            e = max(abs(float(obj.item()) - ref[0]) / abs(ref[0]), rel_l2(gv.cpu().numpy(), ref[1]),
                    rel_l2(gp.cpu().numpy(), ref[2]))
        else:
            e = rel_l2(r.result.cpu().numpy(), ref)
        say(f"  request {r.id} {r.kind} shots {r.geom.nshots} nt {r.grid.nt} merged {r.merged}: {e:.3e}")
        assert e < 1e-4, (r.id, r.kind, e)


def test_serve_tight_budget_waits_and_matches():
    import torch
    from paper_2206_02362_amd.serve import Server, request_bytes
    say("case: 14-request mix, budget = 1.5 x largest request")
    mix = _small_mix(11)
    probe = Server(0, slots=1)
    reqs = serve_setup(mix, probe)
    for r in reqs:
        r.grid = probe.grid_for(r)
    budget = int(1.5 * max(request_bytes(r) for r in reqs))
    srv = Server(0, slots=4, hbm_budget=budget, engine=True, engine_steps=32)
    srv.models = probe.models
    torch.cuda.synchronize()
    srv.replay(reqs, [s.arrival for s in mix.requests])
    torch.cuda.synchronize()
    assert srv.peak_reserved <= budget
    _compare(reqs, _alone(reqs, srv))


def test_serve_full_size_grids_short_time():
    import torch
    from paper_2206_02362_amd.serve import Server
    say("case: request mix on 200x600 .. 600x3000 grids, 1-32 shots, nt capped at 200")
    mix = synth.serve_mix(nreq=8, seed=42)
    srv = Server(0, slots=3, engine=True)
    reqs = serve_setup(mix, srv, nt_cap=200)
    torch.cuda.synchronize()
    srv.replay(reqs, [s.arrival for s in mix.requests])
    torch.cuda.synchronize()
    say("  kinds:", [(r.kind, r.geom.nshots, r.grid.nz, r.grid.nx) for r in reqs])
    _compare(reqs, _alone(reqs, srv))
