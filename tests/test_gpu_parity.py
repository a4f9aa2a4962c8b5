"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: relative L2 <= 1e-4 on traces, images and gradients over the whole
output array, and dot-product error <= 1e-5 with inner products in FP64.
Both sides receive identical inputs (the oracle takes the float32-rounded
arrays as float64).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from _helpers import dot_err, gpu_problem, oracle_problem_f32, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-4
DOT_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2206_02362_amd as fw
    assert torch.cuda.is_available()
    c = fw.Context(0)
    yield c
    c.close()


def t2n(t):
    return t.detach().double().cpu().numpy()


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


# ---------------------------------------------------------------------------
# Nonlinear modeling
# ---------------------------------------------------------------------------

def test_model_tiny_multishot(ctx):
    say("case: model tiny 24x32 nb8 nt160 3 shots")
    w = synth.tiny(nz=24, nx=32, nb=8, nt=160, nshots=3)
    g, geo, vel = oracle_problem_f32(w)
    ref = oracle.model(g, vel, geo)
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.model(grid, tv, tg))
    assert rel_l2(out, ref) < TOL


def test_model_plain_small(ctx):
    say("case: model 100x200 nb40 nt1500 (plain-small)")
    w = synth.plain_small()
    g, geo, vel = oracle_problem_f32(w)
    ref = oracle.model(g, vel, geo)
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.model(grid, tv, tg))
    err = rel_l2(out, ref)
    say("  rel-L2", err)
    assert err < TOL


def test_model_tile_widths_bitwise(ctx):
    # The per-cell arithmetic does not depend on the tile shape.
    import paper_2206_02362_amd as fw
    say("case: model tile widths 16/24/32/48/64")
    w = synth.tiny(nz=70, nx=90, nb=6, nt=120, nshots=2)
    grid, tv, tg = gpu_problem(w)
    outs = []
    old = os.environ.get("FWIME_TILE_X")
    try:
        for tx in ("16", "24", "32", "48", "64"):
            os.environ["FWIME_TILE_X"] = tx
            c = fw.Context(0)
            outs.append(t2n(c.model(grid, tv, tg)))
            c.close()
    finally:
        if old is None:
            os.environ.pop("FWIME_TILE_X", None)
        else:
            os.environ["FWIME_TILE_X"] = old
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_model_shot_alone_equals_in_batch(ctx):
    say("case: model shot alone vs batch")
    w = synth.tiny(nz=40, nx=60, nb=8, nt=150, nshots=4)
    grid, tv, tg = gpu_problem(w)
    full = t2n(ctx.model(grid, tv, tg))
    w1 = w.subset([2])
    grid1, tv1, tg1 = gpu_problem(w1)
    one = t2n(ctx.model(grid1, tv1, tg1))
    assert np.array_equal(full[2], one[0])


def test_model_edge_geometry(ctx):
    # receivers on the model corners, duplicated receivers, no absorbing strip
    say("case: model edge geometry nb0")
    w = synth.tiny(nz=20, nx=30, nb=0, nt=100, nshots=1)
    w.rec_iz = np.array([[0, 0, 19, 19, 5, 5]], np.int32)
    w.rec_ix = np.array([[0, 29, 0, 29, 7, 7]], np.int32)
    w.src_iz[:] = 0
    w.src_ix[:] = 29
    g, geo, vel = oracle_problem_f32(w)
    ref = oracle.model(g, vel, geo)
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.model(grid, tv, tg))
    assert rel_l2(out, ref) < TOL
    assert np.array_equal(out[0, 4], out[0, 5])


# ---------------------------------------------------------------------------
# Extended Born
# ---------------------------------------------------------------------------

def _ptilde(w, seed):
    return synth.random_ptilde(w.nh, w.nz, w.nx, seed).astype(np.float32)


def test_born_ext_fwd_tiny(ctx):
    say("case: born_ext_fwd tiny nh5")
    w = synth.tiny(nz=24, nx=32, nb=8, nt=160, nshots=2, nh=5)
    g, geo, vel = oracle_problem_f32(w)
    pt = _ptilde(w, 3)
    ref = oracle.born_ext_fwd(g, vel, geo, pt.astype(np.float64))
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.born_ext_fwd(grid, tv, tg, dev(pt)))
    assert rel_l2(out, ref) < TOL


def test_born_ext_fwd_offsets_leave_grid(ctx):
    say("case: born_ext_fwd nb3 nh11 (offsets leave the padded grid)")
    w = synth.tiny(nz=12, nx=14, nb=3, nt=90, nshots=1, nh=11)
    g, geo, vel = oracle_problem_f32(w)
    pt = _ptilde(w, 4)
    ref = oracle.born_ext_fwd(g, vel, geo, pt.astype(np.float64))
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.born_ext_fwd(grid, tv, tg, dev(pt)))
    assert rel_l2(out, ref) < TOL


def test_born_ext_fwd_nh1_is_born(ctx):
    say("case: born_ext_fwd nh1")
    w = synth.tiny(nz=24, nx=32, nb=8, nt=160, nshots=2, nh=1)
    g, geo, vel = oracle_problem_f32(w)
    dv = synth.random_ptilde(1, w.nz, w.nx, 5).astype(np.float32)
    dvp = np.zeros((w.nx + 2 * w.nb, w.nz + 2 * w.nb))
    dvp[w.nb:w.nb + w.nx, w.nb:w.nb + w.nz] = dv[0]
    ref = oracle.born(g, vel, geo, dvp)
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.born_ext_fwd(grid, tv, tg, dev(dv)))
    assert rel_l2(out, ref) < TOL


def test_born_ext_fwd_plain_small(ctx):
    say("case: born_ext_fwd 100x200 nt1500 nh11")
    w = synth.plain_small()
    g, geo, vel = oracle_problem_f32(w)
    pt = _ptilde(w, 6)
    ref = oracle.born_ext_fwd(g, vel, geo, pt.astype(np.float64))
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.born_ext_fwd(grid, tv, tg, dev(pt)))
    err = rel_l2(out, ref)
    say("  rel-L2", err)
    assert err < TOL


def _residual_data(w, g, geo, vel):
    # a realistic adjoint source: data of a perturbed model minus data of vel
    pert = vel + 100.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 9, 60.0)
    d = oracle.model(g, pert, geo) - oracle.model(g, vel, geo)
    return d.astype(np.float32)


def test_born_ext_adj_tiny(ctx):
    say("case: born_ext_adj tiny nh5")
    w = synth.tiny(nz=24, nx=32, nb=8, nt=160, nshots=2, nh=5)
    g, geo, vel = oracle_problem_f32(w)
    d = _residual_data(w, g, geo, vel)
    ref = oracle.born_ext_adj(g, vel, geo, d.astype(np.float64), w.nh)
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.born_ext_adj(grid, tv, tg, dev(d), w.nh))
    assert rel_l2(out, ref) < TOL


def test_born_ext_adj_plain_small(ctx):
    say("case: born_ext_adj 100x200 nt1500 nh11")
    w = synth.plain_small()
    g, geo, vel = oracle_problem_f32(w)
    d = _residual_data(w, g, geo, vel)
    ref = oracle.born_ext_adj(g, vel, geo, d.astype(np.float64), w.nh)
    grid, tv, tg = gpu_problem(w)
    out = t2n(ctx.born_ext_adj(grid, tv, tg, dev(d), w.nh))
    err = rel_l2(out, ref)
    say("  rel-L2", err)
    assert err < TOL


def test_dot_product_plain_small(ctx):
    say("case: dot product 100x200 nt1500 nh11")
    w = synth.plain_small()
    grid, tv, tg = gpu_problem(w)
    rng = np.random.default_rng(8)
    pt = rng.standard_normal((w.nh, w.nx, w.nz)).astype(np.float32)
    d = rng.standard_normal((w.nshots, w.nrec, w.nt)).astype(np.float32)
    bp = t2n(ctx.born_ext_fwd(grid, tv, tg, dev(pt)))
    btd = t2n(ctx.born_ext_adj(grid, tv, tg, dev(d), w.nh))
    lhs = float(np.sum(bp * d.astype(np.float64)))
    rhs = float(np.sum(pt.astype(np.float64) * btd))
    # this draw is ill-conditioned: <Fp, d> is 0.074 of its typical size
    # |Fp| |d| / sqrt(N), so the operators' inconsistency is amplified ~13x
    corr = abs(lhs) / (np.linalg.norm(bp) * np.linalg.norm(d)) * np.sqrt(d.size)
    say("  dot err", dot_err(lhs, rhs), "normalized correlation x sqrt(N)", corr)
    assert dot_err(lhs, rhs) < DOT_TOL
    # the same check without the cancellation: d2 = (|d| / |Fp|) Fp + d
    d2 = (bp * (np.linalg.norm(d) / np.linalg.norm(bp)) + d).astype(np.float32)
    lhs2 = float(np.sum(bp * d2.astype(np.float64)))
    rhs2 = float(np.sum(pt.astype(np.float64) * t2n(ctx.born_ext_adj(grid, tv, tg, dev(d2), w.nh))))
    say("  d = Fp-scaled + d: dot err", dot_err(lhs2, rhs2))
    assert dot_err(lhs2, rhs2) < DOT_TOL


@pytest.mark.parametrize("nh", [21, 41, 61])
def test_born_ext_wide_offsets(ctx, nh):
    # offset counts that select the wider scatter and imaging variants
    # (|h| up to 10, 20, 30 cells); 70 x 150 spans two depth strips and a
    # ragged column block
    say(f"case: born_ext_fwd / adj 70x150 nb8 nt120 nh{nh}")
    w = synth.tiny(nz=70, nx=150, nb=8, nt=120, nshots=2, nh=nh, seed=nh)
    g, geo, vel = oracle_problem_f32(w)
    pt = _ptilde(w, nh)
    grid, tv, tg = gpu_problem(w)
    ref = oracle.born_ext_fwd(g, vel, geo, pt.astype(np.float64))
    out = t2n(ctx.born_ext_fwd(grid, tv, tg, dev(pt)))
    e_f = rel_l2(out, ref)
    d = _residual_data(w, g, geo, vel)
    ref = oracle.born_ext_adj(g, vel, geo, d.astype(np.float64), w.nh)
    out = t2n(ctx.born_ext_adj(grid, tv, tg, dev(d), w.nh))
    e_a = rel_l2(out, ref)
    say("  rel-L2 fwd", e_f, "adj", e_a)
    assert e_f < TOL and e_a < TOL


@pytest.fixture(scope="module")
def full_size():
    """The benchmark's offset problem: 300 x 1700 grid, 100 shots, nt = 5000, 61 offsets."""
    w = synth.marmousi_set(100, 17)
    return w, gpu_problem(w)


@pytest.mark.parametrize("seed", [2206, 2207, 2208])
def test_dot_product_full_size(ctx, full_size, seed):
    # The benchmark's own problem in the launch configuration it times, random
    # p and random d drawn per seed.  The relative error is the operator pair's
    # inconsistency divided by the normalized correlation of Fp and d; both
    # are printed.  The d' = (|r| / |Fp|) Fp + r form (no cancellation) is
    # asserted as well.
    import torch
    say(f"case: dot product 300x1700 100 shots nt5000 nh61, seed {seed}")
    w, (grid, tv, tg) = full_size
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    pt = torch.randn((w.nh, w.nx, w.nz), generator=gen, device="cuda:0")
    r = torch.randn((w.nshots, w.nrec, w.nt), generator=gen, device="cuda:0")
    bp = ctx.born_ext_fwd(grid, tv, tg, pt).double()
    nfp, nr = float(bp.norm()), float(r.double().norm())
    assert np.isfinite(nfp) and nfp > 0.0
    lhs_r = float(torch.sum(bp * r.double()))
    rhs_r = float(torch.sum(pt.double() * ctx.born_ext_adj(grid, tv, tg, r, w.nh).double()))
    corr = abs(lhs_r) / (nfp * nr) * np.sqrt(r.numel())
    err_r = dot_err(lhs_r, rhs_r)
    say("  random d: dot err", err_r, "normalized correlation x sqrt(N)", corr)
    d = (bp * (nr / nfp) + r.double()).float()
    lhs = float(torch.sum(bp * d.double()))
    rhs = float(torch.sum(pt.double() * ctx.born_ext_adj(grid, tv, tg, d, w.nh).double()))
    say("  d = Fp-scaled + r: dot err", dot_err(lhs, rhs))
    assert err_r < DOT_TOL
    assert dot_err(lhs, rhs) < DOT_TOL


def test_born_linearity_full_size(ctx):
    # F(a p1 + b p2) = a F p1 + b F p2 on the benchmark's problem (300 x 1700,
    # 100 shots, nt = 5000, 61 offsets): exact in exact arithmetic, so the
    # FP32 difference is rounding only
    import torch
    say("case: born_ext_fwd linearity 300x1700 100 shots nt5000 nh61")
    w = synth.marmousi_set(100, 17)
    grid, tv, tg = gpu_problem(w)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(62)
    p1 = torch.randn((w.nh, w.nx, w.nz), generator=gen, device="cuda:0")
    p2 = torch.randn((w.nh, w.nx, w.nz), generator=gen, device="cuda:0")
    f12 = ctx.born_ext_fwd(grid, tv, tg, 0.75 * p1 - 1.5 * p2).double()
    ref = 0.75 * ctx.born_ext_fwd(grid, tv, tg, p1).double()
    ref -= 1.5 * ctx.born_ext_fwd(grid, tv, tg, p2).double()
    err = float((f12 - ref).norm() / ref.norm())
    say("  rel-L2", err)
    assert np.isfinite(err) and err < TOL


# ---------------------------------------------------------------------------
# FWIME gradient
# ---------------------------------------------------------------------------

def _grad_case(w, seed=0):
    g, geo, vel = oracle_problem_f32(w)
    true = vel + 120.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 40 + seed, 80.0)
    dobs = oracle.model(g, true, geo).astype(np.float32)
    rng = np.random.default_rng(50 + seed)
    pt = (0.2 * rng.standard_normal((w.nh, w.nx, w.nz))).astype(np.float32)
    dso = synth.dso_weights(w.nh)
    return g, geo, vel, dobs, pt, dso


def _check_gradient(ctx, w, eps, seed=0, tol=TOL):
    g, geo, vel, dobs, pt, dso = _grad_case(w, seed)
    obj_r, gv_r, gp_r = oracle.gradient(g, vel, geo, pt.astype(np.float64), dobs.astype(np.float64), eps, dso)
    grid, tv, tg = gpu_problem(w)
    obj, gv, gp = ctx.gradient(grid, tv, tg, dev(pt), dev(dobs), eps, dso)
    e_obj = abs(float(obj.item()) - obj_r) / abs(obj_r)
    e_gv = rel_l2(t2n(gv), gv_r)
    e_gp = rel_l2(t2n(gp), gp_r)
    say("  obj", e_obj, "grad_vel", e_gv, "grad_ptilde", e_gp)
    assert e_obj < tol and e_gv < tol and e_gp < tol


def test_gradient_tiny(ctx):
    say("case: gradient tiny nh5 eps1e-3")
    _check_gradient(ctx, synth.tiny(nz=24, nx=32, nb=8, nt=160, nshots=2, nh=5), 1e-3)


def test_gradient_tiny_eps0(ctx):
    say("case: gradient tiny nh3 eps0")
    _check_gradient(ctx, synth.tiny(nz=20, nx=26, nb=5, nt=130, nshots=1, nh=3), 0.0, seed=1)


def test_gradient_plain_small_600(ctx):
    say("case: gradient 100x200 nt600 nh11")
    w = synth.plain_small()
    w = synth.Workload(w.name, w.nz, w.nx, w.nb, 600, w.dz, w.dx, w.dt, w.vel, w.src_iz, w.src_ix, w.rec_iz,
                       w.rec_ix, w.wavelet[:, :600].copy(), w.nh)
    _check_gradient(ctx, w, 1e-3)


def test_gradient_plain_small_full(ctx):
    # the whole 100 x 200 problem: nt = 1500, 11 offsets (FP32 drift grows with nt)
    say("case: gradient 100x200 nt1500 nh11")
    _check_gradient(ctx, synth.plain_small(), 1e-3)


# ---------------------------------------------------------------------------
# Error paths: nothing is written to the outputs
# ---------------------------------------------------------------------------

def test_errors_leave_outputs_untouched(ctx):
    import torch
    import paper_2206_02362_amd as fw
    say("case: error paths")
    w = synth.tiny(nz=16, nx=20, nb=4, nt=50, nshots=1, nh=3)
    grid, tv, tg = gpu_problem(w)
    data = torch.full((1, w.nrec, w.nt), 7.0, device="cuda:0")
    # CFL violation
    bad = fw.Grid(grid.nz, grid.nx, grid.nb, grid.nt, grid.dz, grid.dx, 0.01)
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_model(bad, tv, tg, data)
    assert e.value.code == fw.FWIME_EINVAL
    # receiver outside the model grid
    rz = w.rec_iz.copy()
    rz[0, 0] = w.nz
    g2 = fw.Geometry(w.src_iz, w.src_ix, rz, w.rec_ix, tg.wavelet)
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_model(grid, tv, g2, data)
    assert e.value.code == fw.FWIME_EINVAL
    # even nh
    pt = torch.zeros((2, w.nx, w.nz), device="cuda:0")
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_born_ext_fwd(grid, tv, tg, 2, pt, data)
    assert e.value.code == fw.FWIME_EINVAL
    # non-finite velocity
    tv2 = tv.clone()
    tv2[3, 3] = float("nan")
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_model(grid, tv2, tg, data)
    assert e.value.code == fw.FWIME_ENONFINITE
    # non-positive velocity
    tv3 = tv.clone()
    tv3[0, 0] = 0.0
    with pytest.raises(fw.FwimeError) as e:
        ctx.fwime_model(grid, tv3, tg, data)
    assert e.value.code == fw.FWIME_EINVAL
    torch.cuda.synchronize()
    assert bool(torch.all(data == 7.0))
