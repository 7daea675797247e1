"""ctypes binding of the FP64 CPU oracle (``lbvp_ref.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. It never imports the HIP library, and the HIP
library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbvp_ref.c")
LIB = os.path.join(HERE, "liblbvp_ref.so")
# a test may point the binding at a deliberately mutated build of the oracle
_LIB_OVERRIDE = os.environ.get("LBVP_REF_LIB")

_SIDE = {"periodic": 0, "inflow_eq": 1, "outflow_zero_grad": 2}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain -O3, OpenMP rows, no FMA contraction)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("tau_plus", C.c_double), ("magic_lambda", C.c_double), ("eta", C.c_double),
                ("rho0", C.c_double),
                ("bc_west", C.c_int32), ("bc_east", C.c_int32), ("bc_south", C.c_int32),
                ("bc_north", C.c_int32),
                ("rho_in", C.c_double), ("u_in_x", C.c_double), ("u_in_y", C.c_double),
                ("fb_x", C.c_double), ("fb_y", C.c_double), ("moving", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            L = C.CDLL(LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        L.lbvp_ref_create.restype = C.c_void_p
        L.lbvp_ref_create.argtypes = [C.POINTER(_Params)]
        L.lbvp_ref_destroy.argtypes = [C.c_void_p]
        L.lbvp_ref_set_mask.argtypes = [C.c_void_p, u8, C.c_int32, C.c_void_p]
        L.lbvp_ref_init_equilibrium.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.lbvp_ref_step.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.lbvp_ref_step_nodes.argtypes = [C.c_void_p, dp, C.c_int64, ip, ip, dp, dp]
        L.lbvp_ref_step_count.restype = C.c_int64
        L.lbvp_ref_step_count.argtypes = [C.c_void_p]
        L.lbvp_ref_set_step_count.argtypes = [C.c_void_p, C.c_int64]
        L.lbvp_ref_read_fields.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        L.lbvp_ref_read_populations.argtypes = [C.c_void_p, dp]
        L.lbvp_ref_write_populations.argtypes = [C.c_void_p, dp]
        L.lbvp_ref_lattice.argtypes = [ip, ip, dp, ip]
        L.lbvp_ref_tau_minus.restype = C.c_double
        L.lbvp_ref_tau_minus.argtypes = [C.c_double, C.c_double]
        L.lbvp_ref_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.lbvp_ref_guo.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.lbvp_ref_trt_collide.argtypes = [dp, dp, dp, C.c_double, C.c_double, dp]
        L.lbvp_ref_vp.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_double,
                                  C.c_double, C.c_double, dp]
        L.lbvp_ref_collide_node.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                            C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.lbvp_ref_num_threads.restype = C.c_int
        L.lbvp_ref_body_at.restype = C.c_int
        L.lbvp_ref_body_at.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64]
        L.lbvp_ref_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------- node pieces --

def lattice() -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    w = np.zeros(9)
    opp = np.zeros(9, np.int32)
    lib().lbvp_ref_lattice(ex, ey, w, opp)
    return ex, ey, w, opp


def tau_minus(tau_plus: float, magic_lambda: float) -> float:
    return lib().lbvp_ref_tau_minus(tau_plus, magic_lambda)


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().lbvp_ref_feq(rho, ux, uy, out)
    return out


def guo(ux: float, uy: float, fx: float, fy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().lbvp_ref_guo(ux, uy, fx, fy, out)
    return out


def trt_collide(f, fe, F, tau_s: float, tau_a: float) -> np.ndarray:
    g = np.zeros(9)
    lib().lbvp_ref_trt_collide(np.ascontiguousarray(f, np.float64), np.ascontiguousarray(fe, np.float64),
                               np.ascontiguousarray(F, np.float64), tau_s, tau_a, g)
    return g


def vp(rho: float, usx: float, usy: float, chi: int, uox: float, uoy: float, eta: float) -> np.ndarray:
    out = np.zeros(4)
    lib().lbvp_ref_vp(rho, usx, usy, int(chi), uox, uoy, eta, out)
    return out


def collide_node(f, tau_s: float, tau_a: float, eta: float, chi: int, uo=(0.0, 0.0), fb=(0.0, 0.0)):
    g = np.zeros(9)
    fl = np.zeros(5)
    lib().lbvp_ref_collide_node(np.ascontiguousarray(f, np.float64), tau_s, tau_a, eta, int(chi),
                                uo[0], uo[1], fb[0], fb[1], g, fl)
    return g, fl


def num_threads() -> int:
    return lib().lbvp_ref_num_threads()


def set_num_threads(n: int) -> None:
    lib().lbvp_ref_set_num_threads(int(n))


# ------------------------------------------------------------------ solver --

class RefSolver:
    """FP64 two-lattice solver over a whole domain (``Problem`` from inputs)."""

    def __init__(self, prob):
        P = _Params(nx=prob.nx, ny=prob.ny, tau_plus=prob.tau_plus, magic_lambda=prob.magic_lambda,
                    eta=prob.eta, rho0=prob.rho0,
                    bc_west=_SIDE[prob.bc[0]], bc_east=_SIDE[prob.bc[1]],
                    bc_south=_SIDE[prob.bc[2]], bc_north=_SIDE[prob.bc[3]],
                    rho_in=prob.rho_in, u_in_x=prob.u_in[0], u_in_y=prob.u_in[1],
                    fb_x=prob.body_force[0], fb_y=prob.body_force[1],
                    moving=1 if getattr(prob, "moving", False) else 0)
        self.nx, self.ny = prob.nx, prob.ny
        self._h = lib().lbvp_ref_create(C.byref(P))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        mask = np.ascontiguousarray(prob.mask_or_empty(), np.uint8)
        bodies = np.ascontiguousarray(prob.bodies_or_empty(), np.float64)
        self.n_bodies = bodies.shape[0]
        if lib().lbvp_ref_set_mask(self._h, mask, self.n_bodies, _ptr(bodies) if self.n_bodies else None):
            raise ValueError("oracle rejected the mask")
        self._keep = (mask, bodies)
        self.init(prob.rho_init, prob.ux_init, prob.uy_init)

    def body_at(self, i: int, j: int, t_level: int) -> int:
        """The mask function chi(x, t) as a body id (moving bodies follow their motion)."""
        return int(lib().lbvp_ref_body_at(self._h, int(i), int(j), int(t_level)))

    def init(self, rho=None, ux=None, uy=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (rho, ux, uy)]
        lib().lbvp_ref_init_equilibrium(self._h, *[_ptr(a) for a in arrs])

    def step(self, n: int = 1, record: bool = False):
        if record:
            forces = np.zeros((n, max(self.n_bodies, 0), 2))
            mass = np.zeros(n)
            lib().lbvp_ref_step(self._h, n, _ptr(forces), _ptr(mass))
            return forces, mass
        lib().lbvp_ref_step(self._h, n, None, None)
        return None

    def step_nodes(self, g: np.ndarray, xs, ys):
        xs = np.ascontiguousarray(xs, np.int32)
        ys = np.ascontiguousarray(ys, np.int32)
        g = np.ascontiguousarray(g, np.float64)
        assert g.shape == (9, self.ny, self.nx)
        gout = np.zeros((len(xs), 9))
        fl = np.zeros((len(xs), 5))
        if lib().lbvp_ref_step_nodes(self._h, g, len(xs), xs, ys, gout, fl):
            raise ValueError("sample outside the grid")
        return gout, fl

    @property
    def step_count(self) -> int:
        return lib().lbvp_ref_step_count(self._h)

    def set_step_count(self, step: int):
        """The state now held (set_populations) is that of time level `step`."""
        if lib().lbvp_ref_set_step_count(self._h, int(step)):
            raise ValueError("step count < 0")

    def fields(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(5)]
        lib().lbvp_ref_read_fields(self._h, *[_ptr(a) for a in out])
        return dict(zip(("rho", "ux", "uy", "fx", "fy"), out))

    def populations(self) -> np.ndarray:
        g = np.zeros((9, self.ny, self.nx))
        lib().lbvp_ref_read_populations(self._h, g)
        return g

    def set_populations(self, g: np.ndarray):
        g = np.ascontiguousarray(g, np.float64)
        assert g.shape == (9, self.ny, self.nx)
        lib().lbvp_ref_write_populations(self._h, g)

    def close(self):
        if self._h:
            lib().lbvp_ref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
