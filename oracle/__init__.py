"""FP64 CPU reference ("the oracle") for the FWIME hot path.

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library neither imports
nor links anything from here, and nothing here imports the GPU library: the
two implementations share no code.  The seeded input generators live in the
separate ``synth`` package, which holds none of the method's arithmetic.

Source of truth: Barnier, Biondi, Clapp and Biondi, "Full waveform inversion
by model extension: practical applications" (arXiv 2206.02362), Section 2
("FWIME theory"): the objective (eq. fwime.obj), the variable-projection
objective (eq. vp.obj) and the gradient split into a Born and a tomographic
part (eqs. fwime.gradient.split, fwime.gradient.born, fwime.gradient.tomo).
The outer loop of Sections 2 and 3 (the linear spline operator S and its
adjoint, L-BFGS with a More-Thuente line search) is in :mod:`oracle.inversion`.
The paper states the operators but not their discretization; every reading
made here is listed in the module docstrings of :mod:`oracle.fd` and
:mod:`oracle.inversion`.
"""
from .fd import (  # noqa: F401
    fd_second_derivative_weights,
    cfl_limit,
    sponge_profile,
    pad_edge,
    pad_edge_adjoint,
    laplacian,
    Grid,
    Geometry,
    model,
    model_adjoint_wavelet,
    born,
    born_adjoint,
    born_ext_fwd,
    born_ext_adj,
    born_ext_tau_fwd,
    born_ext_tau_adj,
    objective,
    gradient,
    vp_objective,
    vp_solve,
)
from .inversion import (  # noqa: F401
    hat_matrix,
    spline_apply,
    spline_adjoint,
    spline_refine,
    two_loop,
    lbfgs,
    on_spline_grid,
)
