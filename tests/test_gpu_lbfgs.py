"""L-BFGS search direction on the GPU (fwime_lbfgs_direction) against the
FP64 oracle's two-loop recursion.

Pairs come from a symmetric positive-definite operator (y = A s), so every
curvature s.y is positive.  Tolerance: relative L2 <= 1e-5 (FP32 vectors,
FP64 inner products); lengths span many 256-thread blocks with a ragged tail.
"""
import sys

import numpy as np
import pytest

import oracle
from _helpers import rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


def _pairs(n, k, seed):
    # A = diag(a) + u u^T with a in [0.5, 20]: SPD, applied without forming it
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 20.0, n)
    u = rng.standard_normal(n) / np.sqrt(n)
    S = rng.standard_normal((k, n)).astype(np.float32)
    Y = np.array([a * s + u * (u @ s) for s in S.astype(np.float64)]).reshape(k, n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    return S, Y, g


@pytest.mark.parametrize("n,k", [(6131, 0), (6131, 1), (6131, 5), (1_000_003, 5), (70_001, 20)])
def test_lbfgs_direction_matches_oracle(ctx, n, k):
    say(f"case: lbfgs direction n {n}, {k} pairs")
    S, Y, g = _pairs(n, k, n + k)
    ref = -oracle.two_loop(g.astype(np.float64), [s.astype(np.float64) for s in S],
                           [y.astype(np.float64) for y in Y])
    out = ctx.lbfgs_direction(dev(S) if k else None, dev(Y) if k else None, dev(g))
    err = rel_l2(out.double().cpu().numpy(), ref)
    say(f"  rel-L2 {err:.3e}")
    assert err < TOL


def test_lbfgs_direction_in_place_and_descent(ctx):
    S, Y, g = _pairs(20_000, 4, 3)
    gd = dev(g)
    d = ctx.lbfgs_direction(dev(S), dev(Y), gd)
    ctx.fwime_lbfgs_direction(dev(S), dev(Y), gd, gd)          # d_out = g
    import torch
    assert torch.equal(d, gd)
    assert float((d.double() * dev(g).double()).sum()) < 0     # H is positive definite


def test_lbfgs_direction_rejects_nonpositive_curvature(ctx):
    import paper_2206_02362_amd as fw
    S, Y, g = _pairs(5000, 3, 9)
    Y[1] = -Y[1]
    out = dev(np.full(5000, 3.0))
    with pytest.raises(fw.FwimeError):
        ctx.fwime_lbfgs_direction(dev(S), dev(Y), dev(g), out)
    assert float(out.min()) == 3.0 and float(out.max()) == 3.0
