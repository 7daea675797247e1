"""Python binding of the D3Q19 entry points of liblbvp.so (include/lbvp3.h), one
function per entry point with the same name, marshalling only. Every step runs
in the library's HIP kernels; there is no CPU fallback (importing raises if the
library is not built).

``Solver3`` wraps a context for a ``Problem3`` (see ``inputs3``) on a torch stream;
``Batch3`` advances several of them together.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import lbvp as _base
from .lbvp import BC, E_ARG, E_DEVICE, E_NOMEM, E_STATE, E_UNSTABLE, GRAPH, KEEP_FIELDS, OK, STORAGE, LbvpError  # noqa: F401

Q = 19
FIELD_NAMES = ("rho", "ux", "uy", "uz", "fx", "fy", "fz")
SYMBOLS = ["lbvp3_footprint_bytes", "lbvp3_create", "lbvp3_set_mask", "lbvp3_init_equilibrium", "lbvp3_step",
           "lbvp3_forces", "lbvp3_read_fields", "lbvp3_read_populations", "lbvp3_write_populations",
           "lbvp3_set_launch", "lbvp3_get_launch", "lbvp3_set_tile_band", "lbvp3_get_tile_band",
           "lbvp3_step_count", "lbvp3_synchronize", "lbvp3_destroy", "lbvp3_save_state", "lbvp3_load_state",
           "lbvp3_last_error", "lbvp3_batch_create", "lbvp3_batch_step", "lbvp3_batch_set_tile_band",
           "lbvp3_batch_get_tile_band", "lbvp3_batch_destroy", "lbvp3_batch_last_error", "lbvp3_tune",
           "lbvp3_tune_last_error"]
NO_STATUS = ("lbvp3_footprint_bytes", "lbvp3_step_count", "lbvp3_last_error", "lbvp3_batch_last_error",
             "lbvp3_tune_last_error")


class lbvp3_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau_plus", C.c_double), ("magic_lambda", C.c_double), ("eta", C.c_double),
                ("rho0", C.c_double), ("bc_west", C.c_int32), ("bc_east", C.c_int32),
                ("rho_in", C.c_double), ("u_in", C.c_double * 3), ("body_force", C.c_double * 3),
                ("storage", C.c_int32), ("force_every", C.c_int32), ("force_capacity", C.c_int64),
                ("max_bodies", C.c_int32), ("flags", C.c_uint32)]


class lbvp3_tune_row(C.Structure):
    _fields_ = [("vec", C.c_int32), ("block", C.c_int32), ("band", C.c_int32),
                ("ms_per_step", C.c_double), ("mlups", C.c_double)]


class lbvp3_body(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("v", C.c_double * 3), ("omega", C.c_double * 3)]


def _load():
    L = _base.lib()
    vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    P = C.POINTER(lbvp3_params)
    L.lbvp3_footprint_bytes.restype = C.c_size_t
    L.lbvp3_footprint_bytes.argtypes = [P]
    L.lbvp3_create.argtypes = [P, vp, C.POINTER(vp)]
    L.lbvp3_set_mask.argtypes = [vp, vp, i32, vp]
    L.lbvp3_init_equilibrium.argtypes = [vp] * 5
    L.lbvp3_step.argtypes = [vp, i64, u32]
    L.lbvp3_forces.argtypes = [vp, vp, vp, i64, C.POINTER(i64), C.POINTER(i64)]
    L.lbvp3_read_fields.argtypes = [vp, i32, i32, vp]
    L.lbvp3_read_populations.argtypes = [vp, i32, i32, vp]
    L.lbvp3_write_populations.argtypes = [vp, i32, i32, vp]
    L.lbvp3_set_launch.argtypes = [vp, i32, i32]
    L.lbvp3_get_launch.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.lbvp3_set_tile_band.argtypes = [vp, i32]
    L.lbvp3_save_state.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    L.lbvp3_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lbvp3_get_tile_band.argtypes = [vp, C.POINTER(i32)]
    L.lbvp3_step_count.restype = i64
    L.lbvp3_step_count.argtypes = [vp]
    L.lbvp3_synchronize.argtypes = [vp]
    L.lbvp3_destroy.argtypes = [vp]
    L.lbvp3_last_error.restype = C.c_char_p
    L.lbvp3_last_error.argtypes = [vp]
    L.lbvp3_batch_create.argtypes = [C.POINTER(vp), i32, i32, i32, C.POINTER(vp)]
    L.lbvp3_batch_step.argtypes = [vp, i64, u32]
    L.lbvp3_batch_set_tile_band.argtypes = [vp, i32]
    L.lbvp3_batch_get_tile_band.argtypes = [vp, C.POINTER(i32)]
    L.lbvp3_batch_destroy.argtypes = [vp]
    L.lbvp3_batch_last_error.restype = C.c_char_p
    L.lbvp3_batch_last_error.argtypes = [vp]
    L.lbvp3_tune.argtypes = [C.POINTER(vp), i32, i32, u32, C.POINTER(lbvp3_tune_row), i32, C.POINTER(i32),
                             C.POINTER(i32)]
    L.lbvp3_tune_last_error.restype = C.c_char_p
    L.lbvp3_tune_last_error.argtypes = []
    for name in SYMBOLS:
        if name not in NO_STATUS:
            getattr(L, name).restype = C.c_int
    return L


_L = _load()


def _ptr(a) -> Optional[int]:
    return None if a is None else a.ctypes.data


def lbvp3_last_error(ctx) -> str:
    msg = _L.lbvp3_last_error(ctx)
    return msg.decode() if msg else ""


def _check(ctx, status: int):
    if status != OK:
        raise LbvpError(status, lbvp3_last_error(ctx))


# ------------------------------------------------------------ the C ABI --

def lbvp3_footprint_bytes(params: lbvp3_params) -> int:
    return int(_L.lbvp3_footprint_bytes(C.byref(params)))


def lbvp3_create(params: lbvp3_params, stream: Optional[int] = None):
    out = C.c_void_p()
    _check(None, _L.lbvp3_create(C.byref(params), stream, C.byref(out)))
    return out.value


def lbvp3_set_mask(ctx, body_id: np.ndarray, bodies: np.ndarray):
    body_id = np.ascontiguousarray(body_id, dtype=np.uint8)
    bodies = np.ascontiguousarray(bodies, dtype=np.float64).reshape(-1, 9)
    n = bodies.shape[0]
    _check(ctx, _L.lbvp3_set_mask(ctx, _ptr(body_id), n, _ptr(bodies) if n else None))


def lbvp3_init_equilibrium(ctx, rho=None, ux=None, uy=None, uz=None):
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, uz)]
    _check(ctx, _L.lbvp3_init_equilibrium(ctx, *[_ptr(a) for a in arrs]))


def lbvp3_step(ctx, n_steps: int, flags: int = 0):
    _check(ctx, _L.lbvp3_step(ctx, int(n_steps), int(flags)))


def lbvp3_forces(ctx, n_bodies: int, cap: int):
    """(forces [n][n_bodies][3], mass [n], first_step); on E_UNSTABLE the filled
    arrays ride on the exception as .data."""
    out = np.zeros((max(cap, 1), max(n_bodies, 1), 3))
    mass = np.zeros(max(cap, 1))
    n, first = C.c_int64(), C.c_int64()
    st = _L.lbvp3_forces(ctx, _ptr(out), _ptr(mass), int(cap), C.byref(n), C.byref(first))
    res = (out[: n.value, :n_bodies].copy(), mass[: n.value].copy(), first.value)
    if st != OK:
        err = LbvpError(st, lbvp3_last_error(ctx))
        err.data = res
        raise err
    return res


def lbvp3_read_fields(ctx, nx: int, ny: int, z0: int, n_planes: int) -> Dict[str, np.ndarray]:
    out = np.zeros((7, n_planes, ny, nx))
    _check(ctx, _L.lbvp3_read_fields(ctx, int(z0), int(n_planes), _ptr(out)))
    return {k: out[q] for q, k in enumerate(FIELD_NAMES)}


def lbvp3_read_populations(ctx, nx: int, ny: int, z0: int, n_planes: int) -> np.ndarray:
    g = np.zeros((Q, n_planes, ny, nx))
    _check(ctx, _L.lbvp3_read_populations(ctx, int(z0), int(n_planes), _ptr(g)))
    return g


def lbvp3_write_populations(ctx, g: np.ndarray, z0: int = 0):
    g = np.ascontiguousarray(g, dtype=np.float64)
    _check(ctx, _L.lbvp3_write_populations(ctx, int(z0), int(g.shape[1]), _ptr(g)))


def lbvp3_set_launch(ctx, vec: int, block: int):
    _check(ctx, _L.lbvp3_set_launch(ctx, int(vec), int(block)))


def lbvp3_get_launch(ctx) -> Tuple[int, int]:
    v, b = C.c_int32(), C.c_int32()
    _check(ctx, _L.lbvp3_get_launch(ctx, C.byref(v), C.byref(b)))
    return v.value, b.value


def lbvp3_set_tile_band(ctx, band: int):
    _check(ctx, _L.lbvp3_set_tile_band(ctx, int(band)))


def lbvp3_get_tile_band(ctx) -> int:
    b = C.c_int32()
    _check(ctx, _L.lbvp3_get_tile_band(ctx, C.byref(b)))
    return b.value


def lbvp3_save_state(ctx) -> np.ndarray:
    """The context's state as a byte array (see lbvp3_save_state)."""
    size = C.c_size_t()
    st = _L.lbvp3_save_state(ctx, None, 0, C.byref(size))
    if st not in (OK, E_NOMEM):
        _check(ctx, st)
    buf = np.empty(size.value, dtype=np.uint8)
    _check(ctx, _L.lbvp3_save_state(ctx, buf.ctypes.data_as(C.c_void_p), buf.nbytes, C.byref(size)))
    return buf


def lbvp3_load_state(ctx, blob):
    blob = np.ascontiguousarray(np.frombuffer(blob, dtype=np.uint8) if isinstance(blob, (bytes, bytearray)) else blob,
                                dtype=np.uint8)
    _check(ctx, _L.lbvp3_load_state(ctx, blob.ctypes.data_as(C.c_void_p), blob.nbytes))


def lbvp3_step_count(ctx) -> int:
    return int(_L.lbvp3_step_count(ctx))


def lbvp3_synchronize(ctx):
    _check(ctx, _L.lbvp3_synchronize(ctx))


def lbvp3_destroy(ctx):
    if ctx:
        _check(None, _L.lbvp3_destroy(ctx))


def lbvp3_batch_last_error(batch) -> str:
    msg = _L.lbvp3_batch_last_error(batch)
    return msg.decode() if msg else ""


def _check_batch(batch, status: int):
    if status != OK:
        raise LbvpError(status, lbvp3_batch_last_error(batch))


def lbvp3_batch_create(ctxs, vec: int = 0, block: int = 0):
    arr = (C.c_void_p * len(ctxs))(*ctxs)
    out = C.c_void_p()
    _check_batch(None, _L.lbvp3_batch_create(arr, len(ctxs), int(vec), int(block), C.byref(out)))
    return out.value


def lbvp3_batch_step(batch, n_steps: int, flags: int = 0):
    _check_batch(batch, _L.lbvp3_batch_step(batch, int(n_steps), int(flags)))


def lbvp3_batch_set_tile_band(batch, band: int):
    _check_batch(batch, _L.lbvp3_batch_set_tile_band(batch, int(band)))


def lbvp3_batch_get_tile_band(batch) -> int:
    b = C.c_int32()
    _check_batch(batch, _L.lbvp3_batch_get_tile_band(batch, C.byref(b)))
    return b.value


def lbvp3_batch_destroy(batch):
    if batch:
        _check_batch(None, _L.lbvp3_batch_destroy(batch))


def lbvp3_tune(ctxs, steps: int = 20, flags: int = 0):
    """(rows as dicts, index of the fastest row)."""
    arr = (C.c_void_p * len(ctxs))(*ctxs)
    cap = 64
    rows = (lbvp3_tune_row * cap)()
    n_rows, best = C.c_int32(), C.c_int32()
    st = _L.lbvp3_tune(arr, len(ctxs), int(steps), int(flags), rows, cap, C.byref(n_rows), C.byref(best))
    if st != OK:
        msg = _L.lbvp3_tune_last_error()
        raise LbvpError(st, msg.decode() if msg else "")
    out = [{"vec": r.vec, "block": r.block, "band": r.band, "ms_per_step": r.ms_per_step, "mlups": r.mlups}
           for r in rows[:min(n_rows.value, cap)]]
    return out, best.value


# ------------------------------------------------------------ convenience --

def params_for(prob, storage: str = "f32", force_every: int = 1, force_capacity: int = 0,
               max_bodies: int = 0) -> lbvp3_params:
    p = lbvp3_params()
    p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
    p.tau_plus, p.magic_lambda, p.eta, p.rho0 = prob.tau_plus, prob.magic_lambda, prob.eta, prob.rho0
    p.bc_west, p.bc_east = (BC[s] for s in prob.bc)
    p.rho_in = prob.rho_in
    for d in range(3):
        p.u_in[d] = prob.u_in[d]
        p.body_force[d] = prob.body_force[d]
    p.storage = STORAGE[storage]
    p.force_every = force_every
    p.force_capacity = force_capacity
    p.max_bodies = max_bodies if max_bodies else max(8, prob.n_bodies)
    p.flags = 0
    return p


class Solver3:
    """A D3Q19 context for one ``Problem3`` on a torch stream."""

    def __init__(self, prob, storage: str = "f32", force_every: int = 1, force_capacity: int = 0,
                 stream: Optional["torch.cuda.Stream"] = None, device: str = "cuda"):
        self.prob = prob
        self.nx, self.ny, self.nz = prob.nx, prob.ny, prob.nz
        self.n_bodies = prob.n_bodies
        self.params = params_for(prob, storage, force_every, force_capacity)
        if lbvp3_footprint_bytes(self.params) == 0:
            raise LbvpError(E_ARG, "invalid parameters")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.ctx = lbvp3_create(self.params, self.stream.cuda_stream)
        lbvp3_set_mask(self.ctx, prob.mask_or_empty(), prob.bodies_or_empty())
        lbvp3_init_equilibrium(self.ctx, prob.rho_init, prob.ux_init, prob.uy_init, prob.uz_init)

    @property
    def footprint(self) -> int:
        return lbvp3_footprint_bytes(self.params)

    def step(self, n: int, keep_fields: bool = False, graph: bool = False):
        lbvp3_step(self.ctx, n, (KEEP_FIELDS if keep_fields else 0) | (GRAPH if graph else 0))

    def forces(self, cap: Optional[int] = None):
        return lbvp3_forces(self.ctx, self.n_bodies, cap or (self.params.force_capacity or 4096))

    def fields(self, z0: int = 0, n_planes: Optional[int] = None) -> Dict[str, np.ndarray]:
        return lbvp3_read_fields(self.ctx, self.nx, self.ny, z0, self.nz - z0 if n_planes is None else n_planes)

    def populations(self, z0: int = 0, n_planes: Optional[int] = None) -> np.ndarray:
        return lbvp3_read_populations(self.ctx, self.nx, self.ny, z0, self.nz - z0 if n_planes is None else n_planes)

    def set_populations(self, g: np.ndarray, z0: int = 0):
        lbvp3_write_populations(self.ctx, g, z0)

    @property
    def step_count(self) -> int:
        return lbvp3_step_count(self.ctx)

    @property
    def launch(self) -> Tuple[int, int]:
        return lbvp3_get_launch(self.ctx)

    def set_launch(self, vec: int, block: int):
        lbvp3_set_launch(self.ctx, vec, block)

    def save_state(self) -> np.ndarray:
        return lbvp3_save_state(self.ctx)

    def load_state(self, blob):
        lbvp3_load_state(self.ctx, blob)

    @property
    def tile_band(self) -> int:
        return lbvp3_get_tile_band(self.ctx)

    def set_tile_band(self, band: int):
        lbvp3_set_tile_band(self.ctx, band)

    def synchronize(self):
        lbvp3_synchronize(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lbvp3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch3:
    """D3Q19 solvers advanced together (one launch per step over all their
    tiles). The solvers must share one stream (pass the same torch stream)."""

    def __init__(self, solvers, vec: int = 0, block: int = 0):
        self.solvers = list(solvers)
        self.handle = lbvp3_batch_create([s.ctx for s in self.solvers], vec, block)

    def step(self, n: int, keep_fields: bool = False, graph: bool = False):
        lbvp3_batch_step(self.handle, n, (KEEP_FIELDS if keep_fields else 0) | (GRAPH if graph else 0))

    @property
    def tile_band(self) -> int:
        return lbvp3_batch_get_tile_band(self.handle)

    def set_tile_band(self, band: int):
        lbvp3_batch_set_tile_band(self.handle, band)

    def close(self):
        if getattr(self, "handle", None):
            lbvp3_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(solvers, steps: int = 20, fresh: bool = False):
    """Time every launch shape and band for these solvers (run together as a
    batch when there are several); returns (rows, best row). The solvers are not
    stepped."""
    rows, best = lbvp3_tune([s.ctx for s in solvers], steps, _base.TUNE_FRESH if fresh else 0)
    return rows, rows[best]
