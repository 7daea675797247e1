"""Python binding of liblbvp.so: the C ABI of include/lbvp.h, one function per
entry point with the same name, marshalling only. Every step of the solver runs
in the library's HIP kernels; there is no CPU fallback. If the library is not
built, importing this module raises.

``Solver`` wraps a context for a ``Problem`` (see ``inputs``): device memory is
a torch uint8 tensor (borrowed by the library) and the stream is a torch stream,
so the caller can time and order the work with torch events.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Tuple

import numpy as np

# torch must load its HIP runtime before liblbvp.so binds to libamdhip64.so.7,
# so that one runtime serves both (streams and pointers are shared).
import torch  # noqa: F401

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbvp.so")

OK, E_ARG, E_NOMEM, E_BUSY, E_DEVICE, E_STATE, E_UNSTABLE = range(7)
STATUS_NAMES = ["OK", "E_ARG", "E_NOMEM", "E_BUSY", "E_DEVICE", "E_STATE", "E_UNSTABLE"]
BC = {"periodic": 0, "inflow_eq": 1, "outflow_zero_grad": 2, "neighbor": 3}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
LAYOUT_AA = 0x1
MOVING_BODIES = 0x2
KEEP_FIELDS = 0x1
GRAPH = 0x2
TUNE_LAYOUTS = 0x1
TUNE_FRESH = 0x2

SYMBOLS = ["lbvp_footprint_bytes", "lbvp_create", "lbvp_set_mask", "lbvp_init_equilibrium",
           "lbvp_step", "lbvp_forces", "lbvp_read_fields", "lbvp_read_populations", "lbvp_read_populations_rows",
           "lbvp_read_fields_rows",
           "lbvp_write_populations", "lbvp_set_launch", "lbvp_get_launch", "lbvp_set_tile_band",
           "lbvp_get_tile_band", "lbvp_step_count",
           "lbvp_synchronize", "lbvp_destroy", "lbvp_last_error", "lbvp_batch_create", "lbvp_batch_step",
           "lbvp_batch_destroy", "lbvp_batch_last_error", "lbvp_tune", "lbvp_tune_last_error",
           "lbvp_pool_create", "lbvp_pool_admit", "lbvp_pool_run_epoch", "lbvp_pool_poll",
           "lbvp_pool_forces", "lbvp_pool_read_fields", "lbvp_pool_release", "lbvp_pool_get_stats",
           "lbvp_pool_destroy", "lbvp_pool_last_error", "lbvp_save_state", "lbvp_load_state",
           "lbvp_device_copy", "lbvp_halo_exchange", "lbvp_batch_set_halo", "lbvp_batch_set_tile_band",
           "lbvp_batch_get_tile_band", "lbvp_batch_step_static"]
NO_STATUS = ("lbvp_footprint_bytes", "lbvp_step_count", "lbvp_last_error", "lbvp_batch_last_error",
             "lbvp_tune_last_error", "lbvp_pool_last_error")


class LbvpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


class lbvp_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("tau_plus", C.c_double), ("magic_lambda", C.c_double), ("eta", C.c_double),
                ("rho0", C.c_double),
                ("bc_west", C.c_int32), ("bc_east", C.c_int32), ("bc_south", C.c_int32),
                ("bc_north", C.c_int32),
                ("rho_in", C.c_double), ("u_in", C.c_double * 2), ("body_force", C.c_double * 2),
                ("storage", C.c_int32), ("force_every", C.c_int32), ("force_capacity", C.c_int64),
                ("max_bodies", C.c_int32), ("flags", C.c_uint32)]


class lbvp_body(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("vx", C.c_double), ("vy", C.c_double),
                ("omega", C.c_double)]


class lbvp_tune_row(C.Structure):
    _fields_ = [("layout_flags", C.c_uint32), ("vec", C.c_int32), ("block", C.c_int32), ("band", C.c_int32),
                ("ms_per_step", C.c_double), ("mlups", C.c_double)]


class lbvp_pool_config(C.Structure):
    _fields_ = [("cap_bytes", C.c_size_t), ("chunk_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("storage", C.c_int32), ("layout_flags", C.c_uint32), ("vec", C.c_int32),
                ("block", C.c_int32), ("max_in_flight", C.c_int32)]


class lbvp_pool_stats(C.Structure):
    _fields_ = [("waiting", C.c_int32), ("running", C.c_int32), ("finished", C.c_int32),
                ("done", C.c_int32), ("free_slots", C.c_int32), ("used_bytes", C.c_size_t),
                ("reserved_bytes", C.c_size_t), ("epochs", C.c_int64), ("node_updates", C.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(or python -m paper_1901_08766_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    P = C.POINTER(lbvp_params)
    L.lbvp_footprint_bytes.restype = C.c_size_t
    L.lbvp_footprint_bytes.argtypes = [P]
    L.lbvp_create.argtypes = [P, vp, vp, C.c_size_t, C.POINTER(vp)]
    L.lbvp_set_mask.argtypes = [vp, vp, i32, vp]
    L.lbvp_init_equilibrium.argtypes = [vp, vp, vp, vp]
    L.lbvp_step.argtypes = [vp, i64, u32]
    L.lbvp_forces.argtypes = [vp, vp, vp, i64, C.POINTER(i64), C.POINTER(i64)]
    L.lbvp_read_fields.argtypes = [vp] * 6
    L.lbvp_read_populations.argtypes = [vp, vp]
    L.lbvp_read_fields_rows.argtypes = [vp, i32, i32] + [vp] * 5
    L.lbvp_read_populations_rows.argtypes = [vp, i32, i32, vp]
    L.lbvp_write_populations.argtypes = [vp, vp]
    L.lbvp_set_launch.argtypes = [vp, i32, i32]
    L.lbvp_get_launch.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.lbvp_set_tile_band.argtypes = [vp, i32]
    L.lbvp_get_tile_band.argtypes = [vp, C.POINTER(i32)]
    L.lbvp_step_count.restype = i64
    L.lbvp_step_count.argtypes = [vp]
    L.lbvp_synchronize.argtypes = [vp]
    L.lbvp_destroy.argtypes = [vp]
    L.lbvp_last_error.restype = C.c_char_p
    L.lbvp_last_error.argtypes = [vp]
    L.lbvp_batch_create.argtypes = [C.POINTER(vp), i32, i32, i32, C.POINTER(vp)]
    L.lbvp_batch_step.argtypes = [vp, i64, u32]
    L.lbvp_batch_destroy.argtypes = [vp]
    L.lbvp_batch_last_error.restype = C.c_char_p
    L.lbvp_batch_last_error.argtypes = [vp]
    L.lbvp_device_copy.argtypes = [vp, vp, C.c_size_t, vp]
    L.lbvp_halo_exchange.argtypes = [C.POINTER(vp), C.POINTER(vp), i32]
    L.lbvp_batch_set_halo.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), i32]
    L.lbvp_batch_step_static.argtypes = [C.POINTER(vp), i32, i64, u32]
    L.lbvp_batch_set_tile_band.argtypes = [vp, i32]
    L.lbvp_batch_get_tile_band.argtypes = [vp, C.POINTER(i32)]
    L.lbvp_save_state.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    L.lbvp_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lbvp_tune.argtypes = [C.POINTER(vp), i32, i32, u32, C.POINTER(lbvp_tune_row), i32, C.POINTER(i32),
                            C.POINTER(i32)]
    L.lbvp_tune_last_error.restype = C.c_char_p
    L.lbvp_tune_last_error.argtypes = []
    L.lbvp_pool_create.argtypes = [C.POINTER(lbvp_pool_config), vp, C.POINTER(vp)]
    L.lbvp_pool_admit.argtypes = [vp, P, vp, i32, vp, vp, vp, vp, i64, C.POINTER(i32)]
    L.lbvp_pool_run_epoch.argtypes = [vp, i64, C.POINTER(i64)]
    L.lbvp_pool_poll.argtypes = [vp, i32, C.POINTER(i32), i32, C.POINTER(i32)]
    L.lbvp_pool_forces.argtypes = [vp, i32, vp, vp, i64, C.POINTER(i64), C.POINTER(i64)]
    L.lbvp_pool_read_fields.argtypes = [vp, i32] + [vp] * 5
    L.lbvp_pool_release.argtypes = [vp, i32]
    L.lbvp_pool_get_stats.argtypes = [vp, C.POINTER(lbvp_pool_stats)]
    L.lbvp_pool_destroy.argtypes = [vp]
    L.lbvp_pool_last_error.restype = C.c_char_p
    L.lbvp_pool_last_error.argtypes = [vp]
    for name in SYMBOLS:
        if name not in NO_STATUS:
            getattr(L, name).restype = C.c_int
    return L


_L = _load()


def lib():
    return _L


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    return a.ctypes.data


def _check(ctx, status: int):
    if status != OK:
        raise LbvpError(status, lbvp_last_error(ctx))


# ------------------------------------------------------------ the C ABI --

def lbvp_last_error(ctx) -> str:
    msg = _L.lbvp_last_error(ctx)
    return msg.decode() if msg else ""


def lbvp_footprint_bytes(params: lbvp_params) -> int:
    return int(_L.lbvp_footprint_bytes(C.byref(params)))


def lbvp_create(params: lbvp_params, stream: Optional[int] = None, dev_mem: Optional[int] = None,
                dev_bytes: int = 0):
    out = C.c_void_p()
    _check(None, _L.lbvp_create(C.byref(params), stream, dev_mem, dev_bytes, C.byref(out)))
    return out.value


def lbvp_set_mask(ctx, body_id: np.ndarray, bodies: np.ndarray):
    body_id = np.ascontiguousarray(body_id, dtype=np.uint8)
    bodies = np.ascontiguousarray(bodies, dtype=np.float64).reshape(-1, 5)
    n = bodies.shape[0]
    _check(ctx, _L.lbvp_set_mask(ctx, _ptr(body_id), n, _ptr(bodies) if n else None))


def lbvp_init_equilibrium(ctx, rho=None, ux=None, uy=None):
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy)]
    _check(ctx, _L.lbvp_init_equilibrium(ctx, *[_ptr(a) for a in arrs]))


def lbvp_step(ctx, n_steps: int, flags: int = 0):
    _check(ctx, _L.lbvp_step(ctx, int(n_steps), int(flags)))


def lbvp_forces(ctx, n_bodies: int, cap: int):
    """Returns (forces [n][n_bodies][2], mass [n], first_step); raises on E_UNSTABLE
    after filling the arrays (they are attached to the exception as .data)."""
    out = np.zeros((max(cap, 1), max(n_bodies, 1), 2))
    mass = np.zeros(max(cap, 1))
    n = C.c_int64()
    first = C.c_int64()
    st = _L.lbvp_forces(ctx, _ptr(out), _ptr(mass), int(cap), C.byref(n), C.byref(first))
    res = (out[: n.value, :n_bodies].copy(), mass[: n.value].copy(), first.value)
    if st != OK:
        err = LbvpError(st, lbvp_last_error(ctx))
        err.data = res
        raise err
    return res


def lbvp_read_fields(ctx, nx: int, ny: int) -> Dict[str, np.ndarray]:
    out = [np.zeros((ny, nx)) for _ in range(5)]
    _check(ctx, _L.lbvp_read_fields(ctx, *[_ptr(a) for a in out]))
    return dict(zip(("rho", "ux", "uy", "fx", "fy"), out))


def lbvp_read_populations(ctx, nx: int, ny: int) -> np.ndarray:
    g = np.zeros((9, ny, nx))
    _check(ctx, _L.lbvp_read_populations(ctx, _ptr(g)))
    return g


def lbvp_read_fields_rows(ctx, nx: int, y0: int, n_rows: int) -> Dict[str, np.ndarray]:
    out = [np.zeros((n_rows, nx)) for _ in range(5)]
    _check(ctx, _L.lbvp_read_fields_rows(ctx, int(y0), int(n_rows), *[_ptr(a) for a in out]))
    return dict(zip(("rho", "ux", "uy", "fx", "fy"), out))


def lbvp_read_populations_rows(ctx, nx: int, y0: int, n_rows: int) -> np.ndarray:
    g = np.zeros((9, n_rows, nx))
    _check(ctx, _L.lbvp_read_populations_rows(ctx, int(y0), int(n_rows), _ptr(g)))
    return g


def lbvp_write_populations(ctx, g: np.ndarray):
    g = np.ascontiguousarray(g, dtype=np.float64)
    _check(ctx, _L.lbvp_write_populations(ctx, _ptr(g)))


def lbvp_device_copy(src: int, dst: int, nbytes: int, stream: Optional[int] = None):
    st = _L.lbvp_device_copy(src, dst, int(nbytes), stream)
    if st != OK:
        raise LbvpError(st, "lbvp_device_copy: pointers and size must be multiples of 16 bytes")


def lbvp_halo_exchange(west, east):
    """One halo exchange over the links (west[i], east[i]) (see lbvp_halo_exchange)."""
    n = len(west)
    w = (C.c_void_p * n)(*west)
    e = (C.c_void_p * n)(*east)
    _check(west[0] if n else None, _L.lbvp_halo_exchange(w, e, n))


def lbvp_save_state(ctx) -> np.ndarray:
    """The context's state as a byte array (see lbvp_save_state)."""
    size = C.c_size_t()
    st = _L.lbvp_save_state(ctx, None, 0, C.byref(size))
    if st not in (OK, E_NOMEM):
        _check(ctx, st)
    buf = np.empty(size.value, dtype=np.uint8)
    _check(ctx, _L.lbvp_save_state(ctx, _ptr(buf), buf.nbytes, C.byref(size)))
    return buf


def lbvp_load_state(ctx, blob):
    blob = np.ascontiguousarray(np.frombuffer(blob, dtype=np.uint8) if isinstance(blob, (bytes, bytearray)) else blob,
                                dtype=np.uint8)
    _check(ctx, _L.lbvp_load_state(ctx, _ptr(blob), blob.nbytes))


def lbvp_set_launch(ctx, vec: int, block: int):
    _check(ctx, _L.lbvp_set_launch(ctx, int(vec), int(block)))


def lbvp_get_launch(ctx) -> Tuple[int, int]:
    v, b = C.c_int32(), C.c_int32()
    _check(ctx, _L.lbvp_get_launch(ctx, C.byref(v), C.byref(b)))
    return v.value, b.value


def lbvp_set_tile_band(ctx, band: int):
    _check(ctx, _L.lbvp_set_tile_band(ctx, int(band)))


def lbvp_get_tile_band(ctx) -> int:
    b = C.c_int32()
    _check(ctx, _L.lbvp_get_tile_band(ctx, C.byref(b)))
    return b.value


def lbvp_step_count(ctx) -> int:
    return int(_L.lbvp_step_count(ctx))


def lbvp_synchronize(ctx):
    _check(ctx, _L.lbvp_synchronize(ctx))


def lbvp_destroy(ctx):
    if ctx:
        _check(None, _L.lbvp_destroy(ctx))


def lbvp_batch_last_error(batch) -> str:
    msg = _L.lbvp_batch_last_error(batch)
    return msg.decode() if msg else ""


def _check_batch(batch, status: int):
    if status != OK:
        raise LbvpError(status, lbvp_batch_last_error(batch))


def lbvp_batch_create(ctxs, vec: int = 0, block: int = 0):
    arr = (C.c_void_p * len(ctxs))(*ctxs)
    out = C.c_void_p()
    _check_batch(None, _L.lbvp_batch_create(arr, len(ctxs), int(vec), int(block), C.byref(out)))
    return out.value


def lbvp_batch_set_halo(batch, west, east):
    n = len(west)
    w = (C.c_int32 * max(n, 1))(*west)
    e = (C.c_int32 * max(n, 1))(*east)
    _check_batch(batch, _L.lbvp_batch_set_halo(batch, w, e, n))


def lbvp_batch_set_tile_band(batch, band: int):
    _check_batch(batch, _L.lbvp_batch_set_tile_band(batch, int(band)))


def lbvp_batch_get_tile_band(batch) -> int:
    b = C.c_int32()
    _check_batch(batch, _L.lbvp_batch_get_tile_band(batch, C.byref(b)))
    return b.value


def lbvp_batch_step(batch, n_steps: int, flags: int = 0):
    _check_batch(batch, _L.lbvp_batch_step(batch, int(n_steps), int(flags)))


def lbvp_batch_step_static(ctxs, n_steps: int, flags: int = 0):
    arr = (C.c_void_p * max(len(ctxs), 1))(*ctxs)
    _check_batch(None, _L.lbvp_batch_step_static(arr, len(ctxs), int(n_steps), int(flags)))


def lbvp_batch_destroy(batch):
    if batch:
        _check_batch(None, _L.lbvp_batch_destroy(batch))


def lbvp_tune_last_error() -> str:
    msg = _L.lbvp_tune_last_error()
    return msg.decode() if msg else ""


def lbvp_tune(ctxs, steps: int, flags: int = 0):
    """Returns (rows, best): rows = [{layout_flags, vec, block, ms_per_step, mlups}]."""
    arr = (C.c_void_p * len(ctxs))(*ctxs)
    cap = 32
    rows = (lbvp_tune_row * cap)()
    n, best = C.c_int32(), C.c_int32()
    st = _L.lbvp_tune(arr, len(ctxs), int(steps), int(flags), rows, cap, C.byref(n), C.byref(best))
    if st != OK:
        raise LbvpError(st, lbvp_tune_last_error())
    out = [{"layout_flags": r.layout_flags, "vec": r.vec, "block": r.block, "band": r.band,
            "ms_per_step": r.ms_per_step, "mlups": r.mlups} for r in rows[: min(n.value, cap)]]
    return out, best.value


def lbvp_pool_last_error(pool) -> str:
    msg = _L.lbvp_pool_last_error(pool)
    return msg.decode() if msg else ""


def _check_pool(pool, status: int):
    if status != OK:
        raise LbvpError(status, lbvp_pool_last_error(pool))


def lbvp_pool_create(cfg: lbvp_pool_config, stream: int):
    out = C.c_void_p()
    _check_pool(None, _L.lbvp_pool_create(C.byref(cfg), stream, C.byref(out)))
    return out.value


def lbvp_pool_admit(pool, params: lbvp_params, body_id: np.ndarray, bodies: np.ndarray, rho=None, ux=None,
                    uy=None, n_steps: int = 1) -> Optional[int]:
    """Slot handle, or None when the pool answers E_BUSY / E_NOMEM (the caller queues)."""
    body_id = np.ascontiguousarray(body_id, dtype=np.uint8)
    bodies = np.ascontiguousarray(bodies, dtype=np.float64).reshape(-1, 5)
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy)]
    slot = C.c_int32()
    nb = bodies.shape[0]
    st = _L.lbvp_pool_admit(pool, C.byref(params), _ptr(body_id), nb, _ptr(bodies) if nb else None,
                            *[_ptr(a) for a in arrs], int(n_steps), C.byref(slot))
    if st in (E_BUSY, E_NOMEM):
        return None
    _check_pool(pool, st)
    return slot.value


def lbvp_pool_run_epoch(pool, max_steps: int) -> int:
    n = C.c_int64()
    _check_pool(pool, _L.lbvp_pool_run_epoch(pool, int(max_steps), C.byref(n)))
    return n.value


def lbvp_pool_poll(pool, wait: bool = False, cap: int = 4096):
    out = (C.c_int32 * cap)()
    n = C.c_int32()
    _check_pool(pool, _L.lbvp_pool_poll(pool, 1 if wait else 0, out, cap, C.byref(n)))
    return list(out[: n.value])


def lbvp_pool_forces(pool, slot: int, n_bodies: int, cap: int):
    out = np.zeros((max(cap, 1), max(n_bodies, 1), 2))
    mass = np.zeros(max(cap, 1))
    n, first = C.c_int64(), C.c_int64()
    st = _L.lbvp_pool_forces(pool, int(slot), _ptr(out), _ptr(mass), int(cap), C.byref(n), C.byref(first))
    res = (out[: n.value, :n_bodies].copy(), mass[: n.value].copy(), first.value)
    if st != OK:
        err = LbvpError(st, lbvp_pool_last_error(pool))
        err.data = res
        raise err
    return res


def lbvp_pool_read_fields(pool, slot: int, nx: int, ny: int) -> Dict[str, np.ndarray]:
    out = [np.zeros((ny, nx)) for _ in range(5)]
    _check_pool(pool, _L.lbvp_pool_read_fields(pool, int(slot), *[_ptr(a) for a in out]))
    return dict(zip(("rho", "ux", "uy", "fx", "fy"), out))


def lbvp_pool_release(pool, slot: int):
    _check_pool(pool, _L.lbvp_pool_release(pool, int(slot)))


def lbvp_pool_get_stats(pool) -> Dict[str, int]:
    s = lbvp_pool_stats()
    _check_pool(pool, _L.lbvp_pool_get_stats(pool, C.byref(s)))
    return {name: getattr(s, name) for name, _ in lbvp_pool_stats._fields_}


def lbvp_pool_destroy(pool):
    if pool:
        _check_pool(None, _L.lbvp_pool_destroy(pool))


# ------------------------------------------------------------ convenience --

def params_for(prob, storage: str = "f32", force_every: int = 1, force_capacity: int = 0,
               max_bodies: int = 0, flags: int = 0) -> lbvp_params:
    p = lbvp_params()
    p.nx, p.ny = prob.nx, prob.ny
    p.tau_plus, p.magic_lambda, p.eta, p.rho0 = prob.tau_plus, prob.magic_lambda, prob.eta, prob.rho0
    p.bc_west, p.bc_east, p.bc_south, p.bc_north = (BC[s] for s in prob.bc)
    p.rho_in = prob.rho_in
    p.u_in[0], p.u_in[1] = prob.u_in
    p.body_force[0], p.body_force[1] = prob.body_force
    p.storage = STORAGE[storage]
    p.force_every = force_every
    p.force_capacity = force_capacity
    p.max_bodies = max_bodies if max_bodies else max(8, prob.n_bodies)
    p.flags = flags | (MOVING_BODIES if getattr(prob, "moving", False) else 0)
    return p


class Solver:
    """A context for one ``Problem``; device memory from torch, stream from torch."""

    def __init__(self, prob, storage: str = "f32", force_every: int = 1, force_capacity: int = 0,
                 flags: int = 0, stream: Optional["torch.cuda.Stream"] = None, device: str = "cuda",
                 mem_fill: Optional[int] = None):
        """mem_fill: a byte value written over the whole device allocation before
        the context is created (0xFF makes every unwritten element a NaN)."""
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        self.n_bodies = prob.n_bodies
        self.params = params_for(prob, storage, force_every, force_capacity, flags=flags)
        nbytes = lbvp_footprint_bytes(self.params)
        if nbytes == 0:
            raise LbvpError(E_ARG, "invalid parameters")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        if mem_fill is not None:
            self.mem.fill_(int(mem_fill))
            torch.cuda.current_stream(self.mem.device).synchronize()
        base = self.mem.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ctx = lbvp_create(self.params, self.stream.cuda_stream, aligned, nbytes)
        lbvp_set_mask(self.ctx, prob.mask_or_empty(), prob.bodies_or_empty())
        lbvp_init_equilibrium(self.ctx, prob.rho_init, prob.ux_init, prob.uy_init)

    @property
    def footprint(self) -> int:
        return lbvp_footprint_bytes(self.params)

    def step(self, n: int, keep_fields: bool = False, graph: bool = False):
        lbvp_step(self.ctx, n, (KEEP_FIELDS if keep_fields else 0) | (GRAPH if graph else 0))

    def forces(self, cap: Optional[int] = None):
        cap = cap or (self.params.force_capacity or 16384)
        return lbvp_forces(self.ctx, self.n_bodies, cap)

    def run(self, n: int, chunk: Optional[int] = None, keep_fields: bool = False):
        """Advance n steps, draining force records as needed; returns
        (forces [records][n_bodies][2], mass [records])."""
        fe = max(self.params.force_every, 1)
        cap = self.params.force_capacity or 16384
        chunk = chunk or max(1, cap * fe)
        fs, ms = [], []
        done = 0
        while done < n:
            k = min(chunk, n - done)
            self.step(k, keep_fields=keep_fields and done + k == n)
            f, m, _ = self.forces()
            fs.append(f)
            ms.append(m)
            done += k
        return np.concatenate(fs) if fs else np.zeros((0, self.n_bodies, 2)), np.concatenate(ms) if ms else np.zeros(0)

    def fields(self, y0: int = 0, n_rows: Optional[int] = None) -> Dict[str, np.ndarray]:
        if y0 == 0 and n_rows is None:
            return lbvp_read_fields(self.ctx, self.nx, self.ny)
        return lbvp_read_fields_rows(self.ctx, self.nx, y0, self.ny - y0 if n_rows is None else n_rows)

    def populations(self, y0: int = 0, n_rows: Optional[int] = None) -> np.ndarray:
        if y0 == 0 and n_rows is None:
            return lbvp_read_populations(self.ctx, self.nx, self.ny)
        return lbvp_read_populations_rows(self.ctx, self.nx, y0, self.ny - y0 if n_rows is None else n_rows)

    def set_populations(self, g: np.ndarray):
        lbvp_write_populations(self.ctx, g)

    def save_state(self) -> np.ndarray:
        return lbvp_save_state(self.ctx)

    def load_state(self, blob):
        lbvp_load_state(self.ctx, blob)

    @property
    def step_count(self) -> int:
        return lbvp_step_count(self.ctx)

    @property
    def launch(self) -> Tuple[int, int]:
        return lbvp_get_launch(self.ctx)

    def set_launch(self, vec: int, block: int):
        lbvp_set_launch(self.ctx, vec, block)

    @property
    def tile_band(self) -> int:
        return lbvp_get_tile_band(self.ctx)

    def set_tile_band(self, band: int):
        lbvp_set_tile_band(self.ctx, band)

    def synchronize(self):
        lbvp_synchronize(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lbvp_destroy(self.ctx)
            self.ctx = None
            self.mem = None   # the context borrowed it; torch may reuse it now

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Solvers advanced together (one launch per step over all their tiles).
    The solvers must share one stream (pass the same torch stream)."""

    def __init__(self, solvers, vec: int = 0, block: int = 0):
        self.solvers = list(solvers)
        self.handle = lbvp_batch_create([s.ctx for s in self.solvers], vec, block)

    def step(self, n: int, keep_fields: bool = False, graph: bool = False):
        lbvp_batch_step(self.handle, n, (KEEP_FIELDS if keep_fields else 0) | (GRAPH if graph else 0))

    @property
    def tile_band(self) -> int:
        return lbvp_batch_get_tile_band(self.handle)

    def set_tile_band(self, band: int):
        lbvp_batch_set_tile_band(self.handle, band)

    def close(self):
        if getattr(self, "handle", None):
            lbvp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(solvers, steps: int = 50, layouts: bool = False, fresh: bool = False):
    """Measure every launch shape (and with ``layouts`` both layouts) for these
    solvers run together; returns (rows, best row). The solvers are not stepped."""
    flags = (TUNE_LAYOUTS if layouts else 0) | (TUNE_FRESH if fresh else 0)
    rows, best = lbvp_tune([s.ctx for s in solvers], steps, flags)
    return rows, rows[best]


class Pool:
    """A serving pool (continuous batching) on one torch stream. ``admit`` takes a
    ``Problem`` and a step count and returns a slot, or None if the pool is full
    now; ``run_epoch`` enqueues one epoch; ``poll`` lists completed slots."""

    def __init__(self, storage: str = "f32", layout_aa: bool = False, cap_bytes: int = 200 * 10**9,
                 max_slots: int = 256, vec: int = 0, block: int = 0, max_in_flight: int = 2,
                 chunk_bytes: int = 0, stream: Optional["torch.cuda.Stream"] = None, device: str = "cuda"):
        self.storage = storage
        self.flags = LAYOUT_AA if layout_aa else 0
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        cfg = lbvp_pool_config()
        cfg.cap_bytes, cfg.chunk_bytes, cfg.max_slots = int(cap_bytes), int(chunk_bytes), int(max_slots)
        cfg.storage, cfg.layout_flags = STORAGE[storage], self.flags
        cfg.vec, cfg.block, cfg.max_in_flight = int(vec), int(block), int(max_in_flight)
        self.handle = lbvp_pool_create(cfg, self.stream.cuda_stream)
        self.probs: Dict[int, object] = {}
        self.steps: Dict[int, int] = {}

    def admit(self, prob, n_steps: int) -> Optional[int]:
        params = params_for(prob, self.storage, 1, 0, flags=self.flags)
        slot = lbvp_pool_admit(self.handle, params, prob.mask_or_empty(), prob.bodies_or_empty(),
                               prob.rho_init, prob.ux_init, prob.uy_init, n_steps)
        if slot is not None:
            self.probs[slot] = prob
            self.steps[slot] = n_steps
        return slot

    def run_epoch(self, max_steps: int) -> int:
        return lbvp_pool_run_epoch(self.handle, max_steps)

    def poll(self, wait: bool = False):
        return lbvp_pool_poll(self.handle, wait)

    def forces(self, slot: int):
        prob = self.probs[slot]
        return lbvp_pool_forces(self.handle, slot, prob.n_bodies, self.steps[slot] + 1)

    def fields(self, slot: int) -> Dict[str, np.ndarray]:
        prob = self.probs[slot]
        return lbvp_pool_read_fields(self.handle, slot, prob.nx, prob.ny)

    def release(self, slot: int):
        lbvp_pool_release(self.handle, slot)
        self.probs.pop(slot, None)
        self.steps.pop(slot, None)

    def stats(self) -> Dict[str, int]:
        return lbvp_pool_get_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            lbvp_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Slabs:
    """One domain decomposed along x into slabs (``inputs.split_x``), each its own
    context with LBVP_BC_NEIGHBOR sides at the cuts, all on one stream. Every
    step is a halo exchange over all cuts, then one step of every slab: batched,
    both run inside lbvp_batch_step (lbvp_batch_set_halo); unbatched, one
    lbvp_halo_exchange and one launch per slab per step. On several GPUs each
    slab would be one GPU's share and the exchange its xGMI transfer; here they
    share one."""

    def __init__(self, slab_problems, x0s, storage: str = "f32", force_every: int = 1, force_capacity: int = 0,
                 batched: bool = True, launch: Optional[Tuple[int, int]] = None, tile_band: Optional[int] = None,
                 stream: Optional["torch.cuda.Stream"] = None, device: str = "cuda", mem_fill: Optional[int] = None):
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.solvers = [Solver(p, storage=storage, force_every=force_every, force_capacity=force_capacity,
                               stream=self.stream, device=device, mem_fill=mem_fill) for p in slab_problems]
        if launch is not None:
            for s in self.solvers:
                s.set_launch(*launch)
        self.x0s = list(x0s)
        n = len(self.solvers)
        # cut k joins slab k's east side to slab k + 1's west side; a periodic
        # domain also joins the last slab to the first
        self.links = [(k, k + 1) for k in range(n - 1)]
        if slab_problems[0].bc[0] == "neighbor":
            self.links.append((n - 1, 0))
        self.batch = Batch(self.solvers, *(launch or (0, 0))) if batched else None
        if self.batch is not None and self.links:   # the exchange runs inside every batched step
            lbvp_batch_set_halo(self.batch.handle, [w for w, _ in self.links], [e for _, e in self.links])
        if tile_band is not None:
            for s in ([self.batch] if self.batch is not None else self.solvers):
                s.set_tile_band(tile_band)

    def exchange(self):
        if self.links:
            lbvp_halo_exchange([self.solvers[w].ctx for w, _ in self.links],
                               [self.solvers[e].ctx for _, e in self.links])

    def step(self, n: int, keep_fields: bool = False, graph: bool = False):
        if self.batch is not None:
            self.batch.step(n, keep_fields=keep_fields, graph=graph)
            return
        for k in range(n):
            self.exchange()
            for s in self.solvers:
                s.step(1, keep_fields=keep_fields and k == n - 1)

    def populations(self) -> np.ndarray:
        return np.concatenate([s.populations() for s in self.solvers], axis=2)

    def fields(self) -> Dict[str, np.ndarray]:
        parts = [s.fields() for s in self.solvers]
        return {k: np.concatenate([p[k] for p in parts], axis=1) for k in parts[0]}

    def forces(self):
        """(force on each body summed over the slabs [records][n_bodies][2],
        mass summed over the slabs [records])."""
        recs = [s.forces() for s in self.solvers]
        return sum(r[0] for r in recs), sum(r[1] for r in recs)

    def close(self):
        if self.batch is not None:
            self.batch.close()
        for s in self.solvers:
            s.close()
