"""ctypes binding of libfwime.so (include/fwime.h): argument marshalling only.

Every numerical step runs in the HIP library.  PyTorch supplies device memory
(tensors) and the stream; the geometry index arrays are host int32 arrays.
There is no fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwime.so")

FWIME_OK = 0
FWIME_EINVAL = 1
FWIME_ENOMEM = 2
FWIME_EHIP = 3
FWIME_ENONFINITE = 4

FWIME_OP_MODEL, FWIME_OP_BORN_FWD, FWIME_OP_BORN_ADJ, FWIME_OP_GRADIENT = 0, 1, 2, 3

EXPORTED = ("fwime_ctx_create", "fwime_ctx_destroy", "fwime_ctx_info", "fwime_ctx_set_timing", "fwime_ctx_trim",
            "fwime_footprint",
            "fwime_model", "fwime_model_static", "fwime_born_ext_fwd",
            "fwime_born_ext_adj", "fwime_born_ext_tau_fwd", "fwime_born_ext_tau_adj", "fwime_gradient", "fwime_gradient_tau", "fwime_vp_solve", "fwime_vp_solve_tau", "fwime_spline_apply", "fwime_spline_adjoint", "fwime_spline_refine", "fwime_lbfgs_direction", "fwime_lbfgs_minimize", "fwime_model_batch", "fwime_engine_create", "fwime_engine_submit", "fwime_engine_run", "fwime_engine_poll",
            "fwime_engine_info", "fwime_engine_destroy", "fwime_forward_tape",
            "fwime_backward_tape", "fwime_tape_free", "fwime_strerror", "fwime_last_error")


# int (*)(void *user, const float *x, float *g, double *f)
OBJECTIVE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_double))
LBFGS_WORK_HEAD = 4096


class FwimeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("nb", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("dz", ctypes.c_double), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("sponge_alpha", ctypes.c_double), ("free_surface", ctypes.c_int32)]


class _Geom(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("src_iz", ctypes.c_void_p), ("src_ix", ctypes.c_void_p),
                ("rec_iz", ctypes.c_void_p), ("rec_ix", ctypes.c_void_p),
                ("wavelet", ctypes.c_void_p)]


class _Job(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("vel", ctypes.c_void_p), ("geom", _Geom), ("data", ctypes.c_void_p)]


class _EngineInfo(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int32), ("active", ctypes.c_int32), ("finishing", ctypes.c_int32),
                ("step", ctypes.c_int64), ("rounds", ctypes.c_int64), ("launches", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("tape_bytes", ctypes.c_size_t), ("tile_x", ctypes.c_int32),
                ("last_batch_tile_x", ctypes.c_int32), ("tuned_signatures", ctypes.c_int32),
                ("last_stencil_launches", ctypes.c_int64), ("last_stencil_ms", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libfwime.so (built in-tree by paper_2206_02362_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2206_02362_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.fwime_ctx_create.argtypes = [I, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.fwime_ctx_create.restype = I
    lib.fwime_ctx_destroy.argtypes = [P]
    lib.fwime_ctx_destroy.restype = None
    lib.fwime_model.argtypes = [P, P, P, P, P, P]
    lib.fwime_model.restype = I
    lib.fwime_model_static.argtypes = [P, P, P, P, P, P]
    lib.fwime_model_static.restype = I
    lib.fwime_born_ext_fwd.argtypes = [P, P, P, P, ctypes.c_int32, P, P, P]
    lib.fwime_born_ext_fwd.restype = I
    lib.fwime_born_ext_adj.argtypes = [P, P, P, P, ctypes.c_int32, P, P, P]
    lib.fwime_born_ext_adj.restype = I
    lib.fwime_born_ext_tau_fwd.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.fwime_born_ext_tau_fwd.restype = I
    lib.fwime_born_ext_tau_adj.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.fwime_born_ext_tau_adj.restype = I
    lib.fwime_gradient.argtypes = [P, P, P, P, ctypes.c_int32, P, P, D, P, P, P, P, P]
    lib.fwime_gradient_tau.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, P, D, P, P, P, P, P]
    lib.fwime_gradient_tau.restype = I
    lib.fwime_vp_solve.restype = I
    lib.fwime_vp_solve.argtypes = [P, P, P, P, ctypes.c_int32, P, D, P, ctypes.c_int32, P, P, P]
    lib.fwime_vp_solve_tau.restype = I
    lib.fwime_vp_solve_tau.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, D, P, ctypes.c_int32, P, P, P]
    lib.fwime_gradient.restype = I
    lib.fwime_lbfgs_minimize.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, D, OBJECTIVE_FN, P,
                                         P, P, ctypes.c_int64, P, P, P]
    lib.fwime_lbfgs_minimize.restype = I
    lib.fwime_lbfgs_direction.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P, P, P, P]
    lib.fwime_lbfgs_direction.restype = I
    lib.fwime_spline_refine.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, P, P, ctypes.c_int32, P,
                                        ctypes.c_int32, P, P, P]
    lib.fwime_spline_refine.restype = I
    for name in ("fwime_spline_apply", "fwime_spline_adjoint"):
        fn = getattr(lib, name)
        fn.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, D, ctypes.c_int32, P, ctypes.c_int32, P, P, P, P]
        fn.restype = I
    lib.fwime_model_batch.argtypes = [P, ctypes.c_int32, P, P]
    lib.fwime_model_batch.restype = I
    lib.fwime_engine_create.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.POINTER(P)]
    lib.fwime_engine_create.restype = I
    lib.fwime_engine_submit.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_int64)]
    lib.fwime_engine_submit.restype = I
    lib.fwime_engine_run.argtypes = [P]
    lib.fwime_engine_run.restype = I
    lib.fwime_engine_poll.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.fwime_engine_poll.restype = I
    lib.fwime_engine_info.argtypes = [P, P]
    lib.fwime_engine_info.restype = I
    lib.fwime_engine_destroy.argtypes = [P]
    lib.fwime_engine_destroy.restype = None
    lib.fwime_ctx_info.argtypes = [P, P]
    lib.fwime_ctx_info.restype = I
    lib.fwime_ctx_set_timing.argtypes = [P, ctypes.c_int32]
    lib.fwime_ctx_set_timing.restype = I
    lib.fwime_ctx_trim.argtypes = [P, P]
    lib.fwime_ctx_trim.restype = I
    lib.fwime_footprint.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_size_t)]
    lib.fwime_footprint.restype = I
    lib.fwime_forward_tape.argtypes = [P, P, P, P, ctypes.c_int32, P, P, ctypes.POINTER(P), P]
    lib.fwime_forward_tape.restype = I
    lib.fwime_backward_tape.argtypes = [P, P, P, P, P, P]
    lib.fwime_backward_tape.restype = I
    lib.fwime_tape_free.argtypes = [P]
    lib.fwime_tape_free.restype = None
    lib.fwime_strerror.argtypes = [I]
    lib.fwime_strerror.restype = ctypes.c_char_p
    lib.fwime_last_error.argtypes = [P]
    lib.fwime_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


@dataclass
class Grid:
    """Model grid (unpadded), absorbing strip and time axis; see fwime_grid_t."""
    nz: int
    nx: int
    nb: int
    nt: int
    dz: float
    dx: float
    dt: float
    sponge_alpha: float = 0.3
    free_surface: bool = False

    def _c(self) -> _Grid:
        return _Grid(self.nz, self.nx, self.nb, self.nt, self.dz, self.dx, self.dt, self.sponge_alpha,
                     1 if self.free_surface else 0)


class Geometry:
    """Acquisition: host int32 index arrays and a device float32 wavelet tensor."""

    def __init__(self, src_iz, src_ix, rec_iz, rec_ix, wavelet: torch.Tensor):
        self.src_iz = np.ascontiguousarray(src_iz, dtype=np.int32)
        self.src_ix = np.ascontiguousarray(src_ix, dtype=np.int32)
        self.rec_iz = np.ascontiguousarray(rec_iz, dtype=np.int32)
        self.rec_ix = np.ascontiguousarray(rec_ix, dtype=np.int32)
        if self.rec_iz.ndim != 2 or self.rec_iz.shape != self.rec_ix.shape:
            raise ValueError("rec_iz / rec_ix must be [nshots][nrec]")
        if self.src_iz.shape != (self.rec_iz.shape[0],) or self.src_ix.shape != self.src_iz.shape:
            raise ValueError("src_iz / src_ix must be [nshots]")
        self.wavelet = wavelet

    @property
    def nshots(self) -> int:
        return int(self.src_iz.shape[0])

    @property
    def nrec(self) -> int:
        return int(self.rec_iz.shape[1])

    def _c(self) -> _Geom:
        return _Geom(self.nshots, self.nrec, self.src_iz.ctypes.data, self.src_ix.ctypes.data,
                     self.rec_iz.ctypes.data, self.rec_ix.ctypes.data, _dptr(self.wavelet, None))


def _dptr(t: torch.Tensor, shape) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"expected float32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Context:
    """Owns a fwime_ctx_t (device scratch arena and HBM budget)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = load()
        self.device = int(device)
        h = ctypes.c_void_p()
        rc = self._lib.fwime_ctx_create(self.device, int(hbm_budget_bytes), ctypes.byref(h))
        if rc != FWIME_OK:
            raise FwimeError(rc, self._lib.fwime_strerror(rc).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fwime_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != FWIME_OK:
            msg = self._lib.fwime_last_error(self._h).decode() or self._lib.fwime_strerror(rc).decode()
            raise FwimeError(rc, msg)

    # --- the four entry points, with caller-provided outputs -----------------
    def fwime_model(self, grid: Grid, vel, geom: Geometry, data):
        g = grid._c()
        ge = geom._c()
        self._check(self._lib.fwime_model(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge),
            _dptr(data, (geom.nshots, geom.nrec, grid.nt)), _stream(vel.device)))

    def fwime_model_static(self, grid: Grid, vel, geom: Geometry, data):
        """fwime_model with its scratch in the library's static device array (no allocation)."""
        g = grid._c()
        ge = geom._c()
        self._check(self._lib.fwime_model_static(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge),
            _dptr(data, (geom.nshots, geom.nrec, grid.nt)), _stream(vel.device)))

    def fwime_born_ext_fwd(self, grid: Grid, vel, geom: Geometry, nh: int, ptilde, data):
        g = grid._c()
        ge = geom._c()
        self._check(self._lib.fwime_born_ext_fwd(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(nh),
            _dptr(ptilde, (nh, grid.nx, grid.nz)), _dptr(data, (geom.nshots, geom.nrec, grid.nt)),
            _stream(vel.device)))

    def fwime_born_ext_adj(self, grid: Grid, vel, geom: Geometry, nh: int, data, ptilde_out):
        g = grid._c()
        ge = geom._c()
        self._check(self._lib.fwime_born_ext_adj(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(nh),
            _dptr(data, (geom.nshots, geom.nrec, grid.nt)), _dptr(ptilde_out, (nh, grid.nx, grid.nz)),
            _stream(vel.device)))

    def fwime_born_ext_tau_fwd(self, grid: Grid, vel, geom: Geometry, ntau: int, lag: int, ptau, data):
        g = grid._c()
        ge = geom._c()
        self._check(self._lib.fwime_born_ext_tau_fwd(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(ntau), int(lag),
            _dptr(ptau, (ntau, grid.nx, grid.nz)), _dptr(data, (geom.nshots, geom.nrec, grid.nt)),
            _stream(vel.device)))

    def fwime_born_ext_tau_adj(self, grid: Grid, vel, geom: Geometry, ntau: int, lag: int, data, ptau_out):
        g = grid._c()
        ge = geom._c()
        self._check(self._lib.fwime_born_ext_tau_adj(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(ntau), int(lag),
            _dptr(data, (geom.nshots, geom.nrec, grid.nt)), _dptr(ptau_out, (ntau, grid.nx, grid.nz)),
            _stream(vel.device)))

    def fwime_gradient(self, grid: Grid, vel, geom: Geometry, nh: int, ptilde, dobs, eps: float, dso,
                       obj, grad_vel, grad_ptilde):
        g = grid._c()
        ge = geom._c()
        dso = np.ascontiguousarray(dso, dtype=np.float64)
        if dso.shape != (nh,):
            raise ValueError("dso must have nh entries")
        if not (isinstance(obj, torch.Tensor) and obj.is_cuda and obj.dtype == torch.float64 and obj.numel() == 1):
            raise TypeError("obj must be a 1-element float64 CUDA tensor")
        self._check(self._lib.fwime_gradient(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(nh),
            _dptr(ptilde, (nh, grid.nx, grid.nz)), _dptr(dobs, (geom.nshots, geom.nrec, grid.nt)),
            float(eps), dso.ctypes.data, obj.data_ptr(), _dptr(grad_vel, (grid.nx, grid.nz)),
            _dptr(grad_ptilde, (nh, grid.nx, grid.nz)), _stream(vel.device)))

    def fwime_gradient_tau(self, grid: Grid, vel, geom: Geometry, ntau: int, lag: int, ptau, dobs, eps: float,
                           dso, obj, grad_vel, grad_ptau):
        g = grid._c()
        ge = geom._c()
        dso = np.ascontiguousarray(dso, dtype=np.float64)
        if dso.shape != (ntau,):
            raise ValueError("dso must have ntau entries")
        if not (isinstance(obj, torch.Tensor) and obj.is_cuda and obj.dtype == torch.float64 and obj.numel() == 1):
            raise TypeError("obj must be a 1-element float64 CUDA tensor")
        self._check(self._lib.fwime_gradient_tau(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(ntau), int(lag),
            _dptr(ptau, (ntau, grid.nx, grid.nz)), _dptr(dobs, (geom.nshots, geom.nrec, grid.nt)),
            float(eps), dso.ctypes.data, obj.data_ptr(), _dptr(grad_vel, (grid.nx, grid.nz)),
            _dptr(grad_ptau, (ntau, grid.nx, grid.nz)), _stream(vel.device)))

    def fwime_vp_solve(self, grid: Grid, vel, geom: Geometry, nh: int, dobs, eps: float, dso, niter: int,
                       ptilde_out):
        """Variable-projection step; returns the objective history (niter + 1 floats)."""
        g = grid._c()
        ge = geom._c()
        dso = np.ascontiguousarray(dso, dtype=np.float64)
        if dso.shape != (nh,):
            raise ValueError("dso must have nh entries")
        if int(niter) < 0:
            raise ValueError("niter must be >= 0")
        phi = np.zeros(int(niter) + 1, dtype=np.float64)
        self._check(self._lib.fwime_vp_solve(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(nh),
            _dptr(dobs, (geom.nshots, geom.nrec, grid.nt)), float(eps), dso.ctypes.data, int(niter),
            _dptr(ptilde_out, (nh, grid.nx, grid.nz)), phi.ctypes.data, _stream(vel.device)))
        return phi

    def fwime_model_batch(self, jobs):
        """jobs: sequence of (Grid, vel, Geometry, data) with caller-provided data tensors."""
        arr = (_Job * len(jobs))()
        keep = []
        stream = None
        for i, (grid, vel, geom, data) in enumerate(jobs):
            arr[i].grid = grid._c()
            arr[i].vel = _dptr(vel, (grid.nx, grid.nz))
            arr[i].geom = geom._c()
            arr[i].data = _dptr(data, (geom.nshots, geom.nrec, grid.nt))
            keep.append(geom)
            stream = _stream(vel.device)
        self._check(self._lib.fwime_model_batch(self._h, len(jobs), ctypes.cast(arr, ctypes.c_void_p), stream))

    def trim(self, stream=None):
        """Release the scratch arena once this context's stream is idle."""
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self._check(self._lib.fwime_ctx_trim(self._h, st))

    def set_timing(self, on: bool = True):
        """Bracket the stencil launch loop of each modeling call with HIP events
        on the call's stream (read back through info())."""
        self._check(self._lib.fwime_ctx_set_timing(self._h, 1 if on else 0))

    def info(self) -> dict:
        out = _Info()
        self._check(self._lib.fwime_ctx_info(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in _Info._fields_}

    def model_batch(self, jobs):
        """jobs: sequence of (Grid, vel, Geometry); returns one data tensor per job."""
        outs = [torch.empty((geom.nshots, geom.nrec, grid.nt), device=vel.device, dtype=torch.float32)
                for grid, vel, geom in jobs]
        self.fwime_model_batch([(g, v, ge, d) for (g, v, ge), d in zip(jobs, outs)])
        return outs

    def fwime_forward_tape(self, grid: Grid, vel, geom: Geometry, nh: int, ptilde, data) -> "Tape":
        g = grid._c()
        ge = geom._c()
        h = ctypes.c_void_p()
        self._check(self._lib.fwime_forward_tape(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(nh),
            _dptr(ptilde, (nh, grid.nx, grid.nz)), _dptr(data, (geom.nshots, geom.nrec, grid.nt)),
            ctypes.byref(h), _stream(vel.device)))
        return Tape(self, h, grid, geom.nshots, geom.nrec, nh, vel.device)

    def fwime_backward_tape(self, tape: "Tape", adjsrc, grad_vel, grad_ptilde):
        g = tape.grid
        self._check(self._lib.fwime_backward_tape(
            self._h, tape._h, _dptr(adjsrc, (tape.nshots, tape.nrec, g.nt)), _dptr(grad_vel, (g.nx, g.nz)),
            _dptr(grad_ptilde, (tape.nh, g.nx, g.nz)), _stream(adjsrc.device)))

    # --- allocating conveniences --------------------------------------------
    def model(self, grid: Grid, vel, geom: Geometry):
        data = torch.empty((geom.nshots, geom.nrec, grid.nt), device=vel.device, dtype=torch.float32)
        self.fwime_model(grid, vel, geom, data)
        return data

    def born_ext_fwd(self, grid: Grid, vel, geom: Geometry, ptilde):
        data = torch.empty((geom.nshots, geom.nrec, grid.nt), device=vel.device, dtype=torch.float32)
        self.fwime_born_ext_fwd(grid, vel, geom, int(ptilde.shape[0]), ptilde, data)
        return data

    def born_ext_adj(self, grid: Grid, vel, geom: Geometry, data, nh: int):
        out = torch.empty((nh, grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        self.fwime_born_ext_adj(grid, vel, geom, nh, data, out)
        return out

    def born_ext_tau_fwd(self, grid: Grid, vel, geom: Geometry, ptau, lag: int):
        data = torch.empty((geom.nshots, geom.nrec, grid.nt), device=vel.device, dtype=torch.float32)
        self.fwime_born_ext_tau_fwd(grid, vel, geom, int(ptau.shape[0]), lag, ptau, data)
        return data

    def born_ext_tau_adj(self, grid: Grid, vel, geom: Geometry, data, ntau: int, lag: int):
        out = torch.empty((ntau, grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        self.fwime_born_ext_tau_adj(grid, vel, geom, ntau, lag, data, out)
        return out

    def gradient(self, grid: Grid, vel, geom: Geometry, ptilde, dobs, eps: float, dso):
        nh = int(ptilde.shape[0])
        obj = torch.empty(1, device=vel.device, dtype=torch.float64)
        gv = torch.empty((grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        gp = torch.empty((nh, grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        self.fwime_gradient(grid, vel, geom, nh, ptilde, dobs, eps, dso, obj, gv, gp)
        return obj, gv, gp


    def gradient_tau(self, grid: Grid, vel, geom: Geometry, ptau, lag: int, dobs, eps: float, dso):
        """(objective, grad_vel, grad_ptau) of eq. fwime.obj with the time-lag extension."""
        ntau = int(ptau.shape[0])
        obj = torch.empty(1, device=vel.device, dtype=torch.float64)
        gv = torch.empty((grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        gp = torch.empty((ntau, grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        self.fwime_gradient_tau(grid, vel, geom, ntau, lag, ptau, dobs, eps, dso, obj, gv, gp)
        return obj, gv, gp

    def fwime_vp_solve_tau(self, grid: Grid, vel, geom: Geometry, ntau: int, lag: int, dobs, eps: float, dso,
                           niter: int, ptau_out):
        """Variable-projection step with time lags; returns the objective history (niter + 1 floats)."""
        g = grid._c()
        ge = geom._c()
        dso = np.ascontiguousarray(dso, dtype=np.float64)
        if dso.shape != (ntau,):
            raise ValueError("dso must have ntau entries")
        if int(niter) < 0:
            raise ValueError("niter must be >= 0")
        phi = np.zeros(int(niter) + 1, dtype=np.float64)
        self._check(self._lib.fwime_vp_solve_tau(
            self._h, ctypes.byref(g), _dptr(vel, (grid.nx, grid.nz)), ctypes.byref(ge), int(ntau), int(lag),
            _dptr(dobs, (geom.nshots, geom.nrec, grid.nt)), float(eps), dso.ctypes.data, int(niter),
            _dptr(ptau_out, (ntau, grid.nx, grid.nz)), phi.ctypes.data, _stream(vel.device)))
        return phi

    def vp_solve_tau(self, grid: Grid, vel, geom: Geometry, dobs, ntau: int, lag: int, eps: float, dso, niter: int):
        """p~ (time lags) after niter CG iterations of the variable-projection step, and the objective history."""
        out = torch.empty((ntau, grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        phi = self.fwime_vp_solve_tau(grid, vel, geom, ntau, lag, dobs, eps, dso, niter, out)
        return out, phi

    def _spline_call(self, fn, nz, nx, dz, dx, zn, xn, src, src_shape, dst, dst_shape):
        zn = np.ascontiguousarray(zn, dtype=np.float64)
        xn = np.ascontiguousarray(xn, dtype=np.float64)
        if zn.ndim != 1 or xn.ndim != 1:
            raise ValueError("node coordinates must be 1D")
        self._check(fn(self._h, int(nz), int(nx), float(dz), float(dx), zn.size, zn.ctypes.data, xn.size,
                       xn.ctypes.data, _dptr(src, src_shape), _dptr(dst, dst_shape), _stream(src.device)))

    def fwime_spline_apply(self, nz: int, nx: int, dz: float, dx: float, zn, xn, mc, out):
        self._spline_call(self._lib.fwime_spline_apply, nz, nx, dz, dx, zn, xn,
                          mc, (len(xn), len(zn)), out, (nx, nz))

    def fwime_spline_adjoint(self, nz: int, nx: int, dz: float, dx: float, zn, xn, f, mc_out):
        self._spline_call(self._lib.fwime_spline_adjoint, nz, nx, dz, dx, zn, xn,
                          f, (nx, nz), mc_out, (len(xn), len(zn)))

    def spline_refine(self, zn, xn, mc, zf, xf):
        """Node values mc [len(xn)][len(zn)] moved to the finer nodes [len(xf)][len(zf)]."""
        zn, xn, zf, xf = (np.ascontiguousarray(v, dtype=np.float64) for v in (zn, xn, zf, xf))
        out = torch.empty((xf.size, zf.size), device=mc.device, dtype=torch.float32)
        self._check(self._lib.fwime_spline_refine(
            self._h, zn.size, zn.ctypes.data, xn.size, xn.ctypes.data, _dptr(mc, (xn.size, zn.size)),
            zf.size, zf.ctypes.data, xf.size, xf.ctypes.data, _dptr(out, None), _stream(mc.device)))
        return out

    def spline_apply(self, nz: int, nx: int, dz: float, dx: float, zn, xn, mc):
        """S m: node values [len(xn)][len(zn)] onto the model grid [nx][nz]."""
        out = torch.empty((nx, nz), device=mc.device, dtype=torch.float32)
        self.fwime_spline_apply(nz, nx, dz, dx, zn, xn, mc, out)
        return out

    def spline_adjoint(self, nz: int, nx: int, dz: float, dx: float, zn, xn, f):
        """S* f: a model-grid field [nx][nz] onto the nodes [len(xn)][len(zn)]."""
        out = torch.empty((len(xn), len(zn)), device=f.device, dtype=torch.float32)
        self.fwime_spline_adjoint(nz, nx, dz, dx, zn, xn, f, out)
        return out

    def fwime_lbfgs_direction(self, s, y, g, d_out):
        n = int(g.numel())
        k = int(s.shape[0]) if s is not None else 0
        sp = _dptr(s, (k, n)) if k else None
        yp = _dptr(y, (k, n)) if k else None
        self._check(self._lib.fwime_lbfgs_direction(self._h, n, k, sp, yp, _dptr(g, (n,)), _dptr(d_out, (n,)),
                                                    _stream(g.device)))

    def lbfgs_direction(self, s, y, g):
        """-H g for the L-BFGS pairs s, y ([k][n], oldest first) and gradient g ([n])."""
        d = torch.empty_like(g)
        self.fwime_lbfgs_direction(s, y, g, d)
        return d

    def lbfgs_minimize(self, fun_grad, x0, memory: int = 5, maxiter: int = 20, gtol: float = 1e-8):
        """L-BFGS from x0 (a float32 device tensor) on fun_grad(x) -> (f, g), with x and g
        device tensors of x0's size; returns (x, f history, iterations)."""
        n = int(x0.numel())
        x = x0.detach().reshape(-1).clone()
        work = torch.empty(LBFGS_WORK_HEAD + (2 * int(memory) + 6) * n, device=x.device, dtype=torch.float32)
        base = work.data_ptr()
        errors = []

        def view(ptr):
            if ptr == x.data_ptr():
                return x
            off = (ptr - base) // 4
            if ptr < base or off + n > work.numel():
                raise RuntimeError("callback pointer outside the workspace")
            return work[off:off + n]

        def callback(user, xp, gp, fp):
            try:
                f, g = fun_grad(view(xp).view_as(x0))
                view(gp).copy_(g.reshape(-1))
                fp[0] = float(f)
                return 0
            except BaseException as e:          # reported after the call returns
                errors.append(e)
                return 1

        cfn = OBJECTIVE_FN(callback)
        hist = np.zeros(int(maxiter) + 1, dtype=np.float64)
        iters = ctypes.c_int32(0)
        rc = self._lib.fwime_lbfgs_minimize(self._h, n, int(memory), int(maxiter), float(gtol), cfn, None,
                                            _dptr(x, (n,)), _dptr(work, None), work.numel(), hist.ctypes.data,
                                            ctypes.byref(iters), _stream(x.device))
        if errors:
            raise errors[0]
        self._check(rc)
        return x.view_as(x0), hist[:iters.value + 1], iters.value

    def vp_solve(self, grid: Grid, vel, geom: Geometry, dobs, nh: int, eps: float, dso, niter: int):
        """p~ after niter CG iterations of the variable-projection step, and the objective history."""
        out = torch.empty((nh, grid.nx, grid.nz), device=vel.device, dtype=torch.float32)
        phi = self.fwime_vp_solve(grid, vel, geom, nh, dobs, eps, dso, niter, out)
        return out, phi


class Engine:
    """Continuous batching of modeling jobs (fwime_engine_*): jobs join a running
    time loop at round boundaries and leave when done.  `stream` is the
    engine's torch stream; every call comes from one host thread."""

    def __init__(self, ctx: Context, stream, steps_per_round: int = 64, max_jobs: int = 256):
        self.ctx = ctx                 # the engine's errors are reported through its context
        self.stream = stream
        h = ctypes.c_void_p()
        ctx._check(ctx._lib.fwime_engine_create(ctx._h, int(steps_per_round), int(max_jobs), stream.cuda_stream,
                                                ctypes.byref(h)))
        self._h = h
        self._jobs = {}                # ticket -> (job struct, geometry, data) kept alive until done

    def submit(self, grid: Grid, vel, geom: Geometry, data, check_stream) -> int:
        """Queue one modeling job writing into `data`; inputs are checked on
        check_stream (where they were written).  Returns its ticket."""
        job = _Job()
        job.grid = grid._c()
        job.vel = _dptr(vel, (grid.nx, grid.nz))
        job.geom = geom._c()
        job.data = _dptr(data, (geom.nshots, geom.nrec, grid.nt))
        t = ctypes.c_int64()
        self.ctx._check(self.ctx._lib.fwime_engine_submit(self._h, ctypes.byref(job), check_stream.cuda_stream,
                                                          ctypes.byref(t)))
        self._jobs[t.value] = (job, geom, vel, data)
        return t.value

    def run(self):
        """Enqueue one round on the engine's stream."""
        self.ctx._check(self.ctx._lib.fwime_engine_run(self._h))

    def poll(self) -> list:
        """Tickets of the jobs whose data is complete."""
        cap = max(1, len(self._jobs))
        buf = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        self.ctx._check(self.ctx._lib.fwime_engine_poll(self._h, ctypes.cast(buf, ctypes.c_void_p), cap,
                                                        ctypes.byref(n)))
        done = [int(buf[i]) for i in range(n.value)]
        for t in done:
            self._jobs.pop(t, None)
        return done

    def info(self) -> dict:
        out = _EngineInfo()
        self.ctx._check(self.ctx._lib.fwime_engine_info(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in _EngineInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.ctx._lib.fwime_engine_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tape:
    """Device-resident checkpoints between fwime_forward_tape and fwime_backward_tape."""

    def __init__(self, ctx: Context, handle, grid: Grid, nshots: int, nrec: int, nh: int, device):
        self.ctx = ctx            # keeps the context alive while the tape exists
        self._h = handle
        self.grid = grid
        self.nshots, self.nrec, self.nh = nshots, nrec, nh
        self.device = device

    def free(self):
        if self._h is not None and self._h.value:
            self.ctx._lib.fwime_tape_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def footprint(grid: Grid, nshots: int, nrec: int, nh: int, op: int) -> int:
    """Device bytes one call of `op` needs to run all shots in one batch."""
    lib = load()
    out = ctypes.c_size_t()
    g = grid._c()
    rc = lib.fwime_footprint(ctypes.byref(g), int(nshots), int(nrec), int(nh), int(op), ctypes.byref(out))
    if rc != FWIME_OK:
        raise FwimeError(rc, lib.fwime_strerror(rc).decode())
    return int(out.value)
