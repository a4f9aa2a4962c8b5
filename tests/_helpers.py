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
