"""Linear spline operator S and its adjoint on the GPU (fwime_spline_apply /
fwime_spline_adjoint) against the FP64 oracle.

Tolerance: relative L2 <= 1e-4 (FP32 weights and sums against FP64); the
dot-product test <S m, f> = <m, S* f> to 1e-5 with inner products in FP64.
Grids span many 256-thread blocks with ragged tails; node sets are uniform,
denser around an interface, and equal to the finite-difference grid (where S
is the identity, bit for bit).
"""
import sys

import numpy as np
import pytest

import oracle
from _helpers import dot_err, rel_l2

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


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def t2n(t):
    return t.detach().double().cpu().numpy()


def _nodes(n, h, every, dense_at=None, seed=0):
    pts = list(np.arange(0, n - 1, every) * h) + [(n - 1) * h]
    if dense_at is not None:
        rng = np.random.default_rng(seed)
        pts += list((dense_at + rng.uniform(-every, every, 6)) * h)
    return np.unique(np.clip(np.array(pts), 0.0, (n - 1) * h))


CASES = [
    # nz, nx, dz, dx, z node spacing (cells), x node spacing, interface row
    (300, 170, 10.0, 10.0, 8, 6, 120),
    (61, 257, 12.5, 25.0, 2, 2, None),        # one halving step away from the grid
    (300, 1700, 10.0, 10.0, 10, 10, 150),     # the benchmark's model size
]


@pytest.mark.parametrize("case", CASES, ids=["300x170", "61x257", "300x1700"])
def test_spline_matches_oracle(ctx, case):
    nz, nx, dz, dx, ez, ex, iface = case
    zn = _nodes(nz, dz, ez, iface, seed=nz)
    xn = _nodes(nx, dx, ex)
    say(f"case: spline apply/adjoint {nz}x{nx}, {len(zn)}x{len(xn)} nodes")
    rng = np.random.default_rng(nz + nx)
    mc = (2000.0 + 300.0 * rng.standard_normal((len(xn), len(zn)))).astype(np.float32)
    f = rng.standard_normal((nx, nz)).astype(np.float32)
    ref = oracle.spline_apply(zn, xn, nz, nx, dz, dx, mc.astype(np.float64))
    out = t2n(ctx.spline_apply(nz, nx, dz, dx, zn, xn, dev(mc)))
    refa = oracle.spline_adjoint(zn, xn, nz, nx, dz, dx, f.astype(np.float64))
    adj = t2n(ctx.spline_adjoint(nz, nx, dz, dx, zn, xn, dev(f)))
    e_f, e_a = rel_l2(out, ref), rel_l2(adj, refa)
    say(f"  rel-L2 apply {e_f:.3e}, adjoint {e_a:.3e}")
    assert e_f < TOL and e_a < TOL


def test_spline_identity_on_the_grid(ctx):
    nz, nx, dz, dx = 77, 301, 10.0, 12.5
    zn, xn = np.arange(nz) * dz, np.arange(nx) * dx
    say("case: spline nodes on the FD grid 77x301")
    f = dev(np.random.default_rng(1).standard_normal((nx, nz)))
    import torch
    assert torch.equal(ctx.spline_apply(nz, nx, dz, dx, zn, xn, f), f)
    assert torch.equal(ctx.spline_adjoint(nz, nx, dz, dx, zn, xn, f), f)


def test_spline_dot_product(ctx):
    nz, nx, dz, dx = 300, 1700, 10.0, 10.0
    zn, xn = _nodes(nz, dz, 7, 100, seed=4), _nodes(nx, dx, 9)
    say(f"case: spline dot product {nz}x{nx}")
    rng = np.random.default_rng(7)
    m = rng.standard_normal((len(xn), len(zn))).astype(np.float32)
    f = rng.standard_normal((nx, nz)).astype(np.float32)
    sm = t2n(ctx.spline_apply(nz, nx, dz, dx, zn, xn, dev(m)))
    sf = t2n(ctx.spline_adjoint(nz, nx, dz, dx, zn, xn, dev(f)))
    lhs = float(np.sum(sm * f.astype(np.float64)))
    rhs = float(np.sum(m.astype(np.float64) * sf))
    say(f"  dot err {dot_err(lhs, rhs):.3e}")
    assert dot_err(lhs, rhs) < DOT_TOL


def test_spline_rejects_bad_nodes(ctx):
    import paper_2206_02362_amd as fw
    nz, nx, dz, dx = 20, 30, 10.0, 10.0
    good_z, good_x = np.array([0.0, 100.0, 190.0]), np.array([0.0, 290.0])
    out = dev(np.full((nx, nz), 7.0))
    bad = [
        (np.array([0.0, 150.0]), good_x),              # does not reach the last depth
        (np.array([5.0, 190.0]), good_x),              # starts below the first point
        (np.array([0.0, 100.0, 100.0, 190.0]), good_x),  # not strictly increasing
        (good_z, np.array([0.0])),                     # one node
        (np.array([0.0, np.nan, 190.0]), good_x),      # not finite
    ]
    for zn, xn in bad:
        mc = dev(np.ones((len(xn), len(zn))))
        with pytest.raises(fw.FwimeError):
            ctx.fwime_spline_apply(nz, nx, dz, dx, zn, xn, mc, out)
    assert float(out.min()) == 7.0 and float(out.max()) == 7.0


def test_spline_refine_matches_oracle(ctx):
    # the next grid of the sequence: every node, every midpoint and a few extra
    # nodes near an interface, on the benchmark's model size
    nz, nx, dz, dx = 300, 1700, 10.0, 10.0
    zn, xn = _nodes(nz, dz, 20, None), _nodes(nx, dx, 20)
    zf = np.unique(np.concatenate([zn, 0.5 * (zn[:-1] + zn[1:]), [1203.7, 1207.1]]))
    xf = np.unique(np.concatenate([xn, 0.5 * (xn[:-1] + xn[1:])]))
    say(f"case: spline refine {len(zn)}x{len(xn)} -> {len(zf)}x{len(xf)} nodes")
    mc = (2000.0 + 300.0 * np.random.default_rng(3).standard_normal((len(xn), len(zn)))).astype(np.float32)
    ref = oracle.spline_refine(zn, xn, mc.astype(np.float64), zf, xf)
    mf = ctx.spline_refine(zn, xn, dev(mc), zf, xf)
    err = rel_l2(t2n(mf), ref)
    # the refined model on the grid is the coarse one
    a = t2n(ctx.spline_apply(nz, nx, dz, dx, zn, xn, dev(mc)))
    b = t2n(ctx.spline_apply(nz, nx, dz, dx, zf, xf, mf))
    say(f"  rel-L2 {err:.3e}, grid models differ by {rel_l2(b, a):.3e}")
    assert err < TOL and rel_l2(b, a) < TOL


def test_spline_refine_rejects_nodes_outside(ctx):
    import paper_2206_02362_amd as fw
    zn, xn = np.array([0.0, 100.0, 200.0]), np.array([0.0, 300.0])
    mc = dev(np.ones((2, 3)))
    for zf in (np.array([0.0, 250.0]), np.array([50.0, 40.0])):
        with pytest.raises(fw.FwimeError):
            ctx.spline_refine(zn, xn, mc, zf, xn)
