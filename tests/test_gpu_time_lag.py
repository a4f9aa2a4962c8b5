"""Extended Born with time lags on the GPU (fwime_born_ext_tau_fwd / _adj)
against the FP64 oracle.

Tolerances as for the offset operators: relative L2 <= 1e-4 on data and
images, dot-product error <= 1e-5 with inner products in FP64.  Lags reach
past both ends of the record (terms dropped), the grids span several tiles
with ragged tails, and one lag reduces to the offset operator with nh = 1.
"""
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
    import paper_2206_02362_amd as fw
    c = fw.Context(0)
    yield c
    c.close()


def t2n(t):
    return t.detach().double().cpu().numpy()


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def _ptau(ntau, w, seed):
    return synth.random_ptilde(ntau, w.nz, w.nx, seed).astype(np.float32)


def _residual_data(w, g, geo, vel):
    pert = vel + 100.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 9, 60.0)
    return (oracle.model(g, pert, geo) - oracle.model(g, vel, geo)).astype(np.float32)


@pytest.mark.parametrize("ntau,lag", [(5, 4), (9, 11), (1, 3)])
def test_time_lag_matches_oracle(ctx, ntau, lag):
    # (9, 11): lags up to 2 * 4 * 11 = 88 steps of a 160-step record
    say(f"case: born_ext_tau fwd/adj 60x90 nb8 nt160 2 shots, ntau {ntau}, lag {lag}")
    w = synth.tiny(nz=60, nx=90, nb=8, nt=160, nshots=2, nh=5, seed=17)
    g, geo, vel = oracle_problem_f32(w)
    grid, tv, tg = gpu_problem(w)
    pt = _ptau(ntau, w, 5)
    ref = oracle.born_ext_tau_fwd(g, vel, geo, pt.astype(np.float64), lag)
    out = t2n(ctx.born_ext_tau_fwd(grid, tv, tg, dev(pt), lag))
    e_f = rel_l2(out, ref)
    d = _residual_data(w, g, geo, vel)
    ref = oracle.born_ext_tau_adj(g, vel, geo, d.astype(np.float64), ntau, lag)
    img = t2n(ctx.born_ext_tau_adj(grid, tv, tg, dev(d), ntau, lag))
    e_a = rel_l2(img, ref)
    say(f"  rel-L2 forward {e_f:.3e}, adjoint {e_a:.3e}")
    assert np.abs(out).max() > 0 and np.abs(img).max() > 0
    assert e_f < TOL and e_a < TOL


@pytest.mark.parametrize("lag,nt", [(1, 300), (2, 400)])
def test_time_lag_101_lags_matches_oracle(ctx, lag, nt):
    # 101 lags (the paper's Marmousi2 count) on a small grid.  lag 1, nt 300:
    # 299 steps / (2 lag) = 150 samples per residue, beyond the LDS kernels'
    # 128, so the direct kernels run; lag 2, nt 400: 100 samples per residue
    # and 50 lags per side, the 64-wide LDS scatter and the 28 / 32-wide LDS
    # imaging kernels
    say(f"case: born_ext_tau fwd/adj 24x32 nb8 nt{nt} 2 shots, ntau 101, lag {lag}")
    ntau = 101
    w = synth.tiny(nz=24, nx=32, nb=8, nt=nt, nshots=2, nh=5, seed=23)
    g, geo, vel = oracle_problem_f32(w)
    grid, tv, tg = gpu_problem(w)
    pt = _ptau(ntau, w, 11)
    ref = oracle.born_ext_tau_fwd(g, vel, geo, pt.astype(np.float64), lag)
    out = t2n(ctx.born_ext_tau_fwd(grid, tv, tg, dev(pt), lag))
    e_f = rel_l2(out, ref)
    d = _residual_data(w, g, geo, vel)
    ref = oracle.born_ext_tau_adj(g, vel, geo, d.astype(np.float64), ntau, lag)
    img = t2n(ctx.born_ext_tau_adj(grid, tv, tg, dev(d), ntau, lag))
    e_a = rel_l2(img, ref)
    say(f"  rel-L2 forward {e_f:.3e}, adjoint {e_a:.3e}")
    assert np.abs(out).max() > 0 and np.abs(img).max() > 0
    assert e_f < TOL and e_a < TOL


def test_time_lag_single_lag_is_offset_operator(ctx):
    # ntau = 1 and nh = 1 build the same scattering source with the same
    # arithmetic and drive the same propagation
    say("case: born_ext_tau ntau 1 against born_ext nh 1, 40x70 nt200")
    w = synth.tiny(nz=40, nx=70, nb=8, nt=200, nshots=2, nh=1, seed=3)
    grid, tv, tg = gpu_problem(w)
    pt = dev(_ptau(1, w, 7))
    a = t2n(ctx.born_ext_tau_fwd(grid, tv, tg, pt, 5))
    b = t2n(ctx.born_ext_fwd(grid, tv, tg, pt))
    say(f"  max |diff| {np.abs(a - b).max():.3e} of max |x| {np.abs(b).max():.3e}")
    assert np.abs(b).max() > 0 and rel_l2(a, b) < 1e-6


def test_time_lag_dot_product(ctx):
    say("case: born_ext_tau dot product 60x90 nt300 ntau 11 lag 6")
    w = synth.tiny(nz=60, nx=90, nb=8, nt=300, nshots=2, nh=5, seed=29)
    grid, tv, tg = gpu_problem(w)
    rng = np.random.default_rng(31)
    ntau, lag = 11, 6
    pt = rng.standard_normal((ntau, w.nx, w.nz)).astype(np.float32)
    d = rng.standard_normal((w.nshots, w.nrec, w.nt)).astype(np.float32)
    bp = t2n(ctx.born_ext_tau_fwd(grid, tv, tg, dev(pt), lag))
    for name, dd in (("random d", d), ("d = Fp-scaled + d", bp * (np.linalg.norm(d) / np.linalg.norm(bp)) + d)):
        dd = dd.astype(np.float32)
        lhs = float(np.sum(bp * dd.astype(np.float64)))
        rhs = float(np.sum(pt.astype(np.float64) * t2n(ctx.born_ext_tau_adj(grid, tv, tg, dev(dd), ntau, lag))))
        say(f"  {name}: dot err {dot_err(lhs, rhs):.3e}")
        assert dot_err(lhs, rhs) < DOT_TOL


def test_time_lag_batches_agree(ctx):
    # a budget that holds one shot's history at a time splits the shots into
    # batches: data identical, images equal up to the order of the shot sums
    import paper_2206_02362_amd as fw
    say("case: born_ext_tau with one shot per batch, 40x70 nt200 3 shots")
    w = synth.tiny(nz=40, nx=70, nb=8, nt=200, nshots=3, nh=5, seed=41)
    grid, tv, tg = gpu_problem(w)
    pt = dev(_ptau(5, w, 2))
    d0 = ctx.born_ext_tau_fwd(grid, tv, tg, pt, 4)
    i0 = t2n(ctx.born_ext_tau_adj(grid, tv, tg, d0, 5, 4))
    # one shot's share of the forward call: 2 (nt - 1) + 10 padded fields
    # ([nx + 2 nb][roundup(nz + 2 nb + 4, 64)] floats) plus its receiver tables
    field = (w.nx + 2 * w.nb) * ((w.nz + 2 * w.nb + 4 + 63) // 64 * 64)
    per_shot = (2 * (w.nt - 1) + 10) * field * 4 + w.nrec * 64
    small = fw.Context(0, hbm_budget_bytes=int(1.5 * per_shot) + (4 << 20))
    d1 = small.born_ext_tau_fwd(grid, tv, tg, pt, 4)
    i1 = t2n(small.born_ext_tau_adj(grid, tv, tg, d1, 5, 4))
    small.close()
    assert np.array_equal(t2n(d0), t2n(d1))
    assert rel_l2(i1, i0) < 1e-6


def test_time_lag_rejects_bad_arguments(ctx):
    import paper_2206_02362_amd as fw
    w = synth.tiny(nz=24, nx=32, nb=8, nt=100, nshots=1, nh=5)
    grid, tv, tg = gpu_problem(w)
    pt = dev(_ptau(5, w, 1))
    for ntau, lag in ((4, 2), (5, 0), (5, 1000)):
        with pytest.raises(fw.FwimeError):
            ctx.fwime_born_ext_tau_fwd(grid, tv, tg, ntau, lag, pt[:ntau] if ntau <= 5 else pt,
                                       dev(np.zeros((1, w.nrec, w.nt))))


def test_time_lag_full_size_dot_product(ctx):
    # the benchmark's setting (300 x 1700, nt 5000, 101 lags of 20 steps), 2
    # shots: a property that holds at any size, since the oracle cannot run here
    import torch
    say("case: born_ext_tau dot product 300x1700 nt5000 ntau 101 lag 20, 2 shots")
    w = synth.marmousi_set(2, 17)
    grid, tv, tg = gpu_problem(w)
    ntau, lag = 101, 20
    g = torch.Generator(device="cuda:0").manual_seed(5)
    pt = torch.randn((ntau, w.nx, w.nz), generator=g, device="cuda:0", dtype=torch.float32)
    d = torch.randn((w.nshots, w.nrec, w.nt), generator=g, device="cuda:0", dtype=torch.float32)
    bp = ctx.born_ext_tau_fwd(grid, tv, tg, pt, lag)
    d2 = bp * (d.norm() / bp.norm()) + d
    for name, dd in (("random d", d), ("d = Fp-scaled + d", d2)):
        lhs = float((bp.double() * dd.double()).sum())
        rhs = float((pt.double() * ctx.born_ext_tau_adj(grid, tv, tg, dd.contiguous(), ntau, lag).double()).sum())
        say(f"  {name}: dot err {dot_err(lhs, rhs):.3e}")
        assert dot_err(lhs, rhs) < DOT_TOL


@pytest.mark.parametrize("ntau,lag,eps", [(5, 4, 1e-3), (9, 7, 0.0), (1, 3, 1e-3)])
def test_time_lag_gradient_matches_oracle(ctx, ntau, lag, eps):
    # objective and both gradients of eq. fwime.obj with the time-lag
    # extension (oracle.gradient with lag=L); (9, 7): lags up to 56 steps of
    # a 170-step record
    say(f"case: gradient_tau 30x44 nb8 nt170 2 shots, ntau {ntau}, lag {lag}, eps {eps}")
    w = synth.tiny(nz=30, nx=44, nb=8, nt=170, nshots=2, nh=5, seed=37)
    g, geo, vel = oracle_problem_f32(w)
    true = vel + 120.0 * synth.gaussian_perturbation(w.nz, w.nx, w.dx, 40, 80.0)
    dobs = oracle.model(g, true, geo).astype(np.float32)
    pt = (0.2 * np.random.default_rng(51).standard_normal((ntau, w.nx, w.nz))).astype(np.float32)
    dso = synth.dso_weights(ntau)
    obj_r, gv_r, gp_r = oracle.gradient(g, vel, geo, pt.astype(np.float64), dobs.astype(np.float64), eps, dso,
                                        lag=lag)
    grid, tv, tg = gpu_problem(w)
    obj, gv, gp = ctx.gradient_tau(grid, tv, tg, dev(pt), lag, dev(dobs), eps, dso)
    e_obj = abs(float(obj.item()) - obj_r) / abs(obj_r)
    e_gv, e_gp = rel_l2(t2n(gv), gv_r), rel_l2(t2n(gp), gp_r)
    say(f"  obj {e_obj:.3e} grad_vel {e_gv:.3e} grad_ptau {e_gp:.3e}")
    assert e_obj < TOL and e_gv < TOL and e_gp < TOL


def test_time_lag_gradient_single_lag_is_offset_gradient(ctx):
    # one lag and one offset build the same objective and gradients
    say("case: gradient_tau ntau 1 against gradient nh 1, 40x60 nt200")
    w = synth.tiny(nz=40, nx=60, nb=8, nt=200, nshots=2, nh=1, seed=43)
    grid, tv, tg = gpu_problem(w)
    pt = dev(0.1 * synth.random_ptilde(1, w.nz, w.nx, 3))
    dobs = dev(0.01 * np.random.default_rng(3).standard_normal((w.nshots, w.nrec, w.nt)))
    a = ctx.gradient_tau(grid, tv, tg, pt, 5, dobs, 1e-3, np.ones(1))
    b = ctx.gradient(grid, tv, tg, pt, dobs, 1e-3, np.ones(1))
    for x, y, name in zip(a, b, ("obj", "grad_vel", "grad_ptau")):
        e = rel_l2(t2n(x), t2n(y))
        say(f"  {name}: rel-L2 {e:.3e}")
        assert e < 1e-5, name
