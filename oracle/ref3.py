"""ctypes binding of the FP64 D3Q19 CPU oracle (``lbvp3_ref.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. It never imports the HIP library, and the HIP
library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbvp3_ref.c")
LIB = os.path.join(HERE, "liblbvp3_ref.so")
# a test may point the binding at a deliberately mutated build of the oracle
_LIB_OVERRIDE = os.environ.get("LBVP3_REF_LIB")

_SIDE = {"periodic": 0, "inflow_eq": 1, "outflow_zero_grad": 2}
Q = 19
FIELD_NAMES = ("rho", "ux", "uy", "uz", "fx", "fy", "fz")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain -O3, OpenMP planes, no FMA contraction)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau_plus", C.c_double), ("magic_lambda", C.c_double), ("eta", C.c_double),
                ("rho0", C.c_double), ("bc_west", C.c_int32), ("bc_east", C.c_int32),
                ("rho_in", C.c_double), ("u_in", C.c_double * 3), ("fb", C.c_double * 3)]


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
        L.lbvp3_ref_create.restype = C.c_void_p
        L.lbvp3_ref_create.argtypes = [C.POINTER(_Params)]
        L.lbvp3_ref_destroy.argtypes = [C.c_void_p]
        L.lbvp3_ref_set_mask.argtypes = [C.c_void_p, u8, C.c_int32, C.c_void_p]
        L.lbvp3_ref_init_equilibrium.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.lbvp3_ref_step.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.lbvp3_ref_step_nodes.argtypes = [C.c_void_p, dp, C.c_int64, ip, ip, ip, dp, dp]
        L.lbvp3_ref_step_count.restype = C.c_int64
        L.lbvp3_ref_step_count.argtypes = [C.c_void_p]
        L.lbvp3_ref_read_fields.argtypes = [C.c_void_p, dp]
        L.lbvp3_ref_read_populations.argtypes = [C.c_void_p, dp]
        L.lbvp3_ref_write_populations.argtypes = [C.c_void_p, dp]
        L.lbvp3_ref_lattice.argtypes = [ip, ip, ip, dp, ip]
        L.lbvp3_ref_feq.argtypes = [C.c_double, dp, dp]
        L.lbvp3_ref_guo.argtypes = [dp, dp, dp]
        L.lbvp3_ref_trt_collide.argtypes = [dp, dp, dp, C.c_double, C.c_double, dp]
        L.lbvp3_ref_collide_node.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, dp, dp]
        L.lbvp3_ref_num_threads.restype = C.c_int
        L.lbvp3_ref_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _v3(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, np.float64).reshape(3))


# ------------------------------------------------------------- node pieces --

def lattice() -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    ex, ey, ez, opp = (np.zeros(Q, np.int32) for _ in range(4))
    w = np.zeros(Q)
    lib().lbvp3_ref_lattice(ex, ey, ez, w, opp)
    return ex, ey, ez, w, opp


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(Q)
    lib().lbvp3_ref_feq(rho, _v3(u), out)
    return out


def guo(u, F) -> np.ndarray:
    out = np.zeros(Q)
    lib().lbvp3_ref_guo(_v3(u), _v3(F), out)
    return out


def trt_collide(f, fe, F, tau_s: float, tau_a: float) -> np.ndarray:
    g = np.zeros(Q)
    lib().lbvp3_ref_trt_collide(np.ascontiguousarray(f, np.float64), np.ascontiguousarray(fe, np.float64),
                                np.ascontiguousarray(F, np.float64), tau_s, tau_a, g)
    return g


def collide_node(f, tau_s: float, tau_a: float, eta: float, chi: int, uo=(0.0, 0.0, 0.0), fb=(0.0, 0.0, 0.0)):
    g = np.zeros(Q)
    fl = np.zeros(7)
    lib().lbvp3_ref_collide_node(np.ascontiguousarray(f, np.float64), tau_s, tau_a, eta, int(chi), _v3(uo),
                                 _v3(fb), g, fl)
    return g, fl


def num_threads() -> int:
    return lib().lbvp3_ref_num_threads()


def set_num_threads(n: int) -> None:
    lib().lbvp3_ref_set_num_threads(int(n))


# ------------------------------------------------------------------ solver --

class RefSolver3:
    """FP64 two-lattice D3Q19 solver over a whole domain (``Problem3``)."""

    def __init__(self, prob):
        P = _Params(nx=prob.nx, ny=prob.ny, nz=prob.nz, tau_plus=prob.tau_plus,
                    magic_lambda=prob.magic_lambda, eta=prob.eta, rho0=prob.rho0,
                    bc_west=_SIDE[prob.bc[0]], bc_east=_SIDE[prob.bc[1]], rho_in=prob.rho_in,
                    u_in=(C.c_double * 3)(*prob.u_in), fb=(C.c_double * 3)(*prob.body_force))
        self.nx, self.ny, self.nz = prob.nx, prob.ny, prob.nz
        self.n = prob.nx * prob.ny * prob.nz
        self._h = lib().lbvp3_ref_create(C.byref(P))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        mask = np.ascontiguousarray(prob.mask_or_empty(), np.uint8)
        bodies = np.ascontiguousarray(prob.bodies_or_empty(), np.float64)
        self.n_bodies = bodies.shape[0]
        if lib().lbvp3_ref_set_mask(self._h, mask, self.n_bodies, _ptr(bodies) if self.n_bodies else None):
            raise ValueError("oracle rejected the mask")
        self._keep = (mask, bodies)
        self.init(prob.rho_init, prob.ux_init, prob.uy_init, prob.uz_init)

    def init(self, rho=None, ux=None, uy=None, uz=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (rho, ux, uy, uz)]
        lib().lbvp3_ref_init_equilibrium(self._h, *[_ptr(a) for a in arrs])

    def step(self, n: int = 1, record: bool = False):
        if record:
            forces = np.zeros((n, self.n_bodies, 3))
            mass = np.zeros(n)
            lib().lbvp3_ref_step(self._h, n, _ptr(forces), _ptr(mass))
            return forces, mass
        lib().lbvp3_ref_step(self._h, n, None, None)
        return None

    def step_nodes(self, g: np.ndarray, xs, ys, zs):
        """One step at the given nodes from populations g [19, nz, ny, nx]."""
        xs, ys, zs = (np.ascontiguousarray(a, np.int32) for a in (xs, ys, zs))
        g = np.ascontiguousarray(g, np.float64)
        assert g.shape == (Q, self.nz, self.ny, self.nx)
        gout = np.zeros((len(xs), Q))
        fl = np.zeros((len(xs), 7))
        if lib().lbvp3_ref_step_nodes(self._h, g, len(xs), xs, ys, zs, gout, fl):
            raise ValueError("node outside the grid")
        return gout, fl

    @property
    def step_count(self) -> int:
        return int(lib().lbvp3_ref_step_count(self._h))

    def fields(self) -> Dict[str, np.ndarray]:
        out = np.zeros((7, self.nz, self.ny, self.nx))
        lib().lbvp3_ref_read_fields(self._h, out)
        return {k: out[q] for q, k in enumerate(FIELD_NAMES)}

    def populations(self) -> np.ndarray:
        g = np.zeros((Q, self.nz, self.ny, self.nx))
        lib().lbvp3_ref_read_populations(self._h, g)
        return g

    def set_populations(self, g: np.ndarray) -> None:
        g = np.ascontiguousarray(g, np.float64)
        assert g.shape == (Q, self.nz, self.ny, self.nx)
        lib().lbvp3_ref_write_populations(self._h, g)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            lib().lbvp3_ref_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: the module may already be gone
            pass
