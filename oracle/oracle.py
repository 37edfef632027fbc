"""ctypes binding of the plain C oracle (``lbsc_oracle.c``).

Test infrastructure only. Arrays are numpy float64. Populations use the layout
``f[c, i, z, y, x]``: component ``c`` (0 = A, the component held at rho_H by
the evaporation sink; 1 = B), direction ``i`` (0 rest, 1-6 axis, 7-18 face
diagonals), then the node in z-major order.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbsc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblbsc_oracle.so")
_lock = threading.Lock()
_lib = None

PSI_RHO, PSI_EXP = 0, 1
SINK_NONE, SINK_ZMAX, SINK_FACES, SINK_SPHERE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over independent per-node loops)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=gnu11", "-O3", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("wall_z", ctypes.c_int),
        ("tau", ctypes.c_double * 2),
        ("g", ctypes.c_double),
        ("psi_kind", ctypes.c_int),
        ("sink_kind", ctypes.c_int),
        ("rho_h", ctypes.c_double),
        ("sink_radius", ctypes.c_double),
        ("center", ctypes.c_double * 3),
        ("phi_delta", ctypes.c_double * 2),
        ("solid_z", ctypes.c_int),
        ("wall_rho", ctypes.c_double * 2),
        ("ncomp", ctypes.c_int),
    ]


class _Diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_longlong),
        ("mass", ctypes.c_double * 2),
        ("evaporated", ctypes.c_double),
        ("evap_rate", ctypes.c_double),
        ("momentum", ctypes.c_double * 3),
        ("z_interface", ctypes.c_double),
        ("r_droplet", ctypes.c_double),
        ("nonfinite", ctypes.c_longlong),
        ("nonpositive", ctypes.c_longlong),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_create.restype = ctypes.c_void_p
        lib.orc_create.argtypes = [ctypes.POINTER(_Params)]
        lib.orc_destroy.argtypes = [ctypes.c_void_p]
        lib.orc_init_from_density.argtypes = [ctypes.c_void_p, dp, dp]
        lib.orc_init_from_populations.argtypes = [ctypes.c_void_p, dp]
        lib.orc_set_sink.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_longlong]
        lib.orc_get_populations.argtypes = [ctypes.c_void_p, dp]
        lib.orc_get_density.argtypes = [ctypes.c_void_p, dp, dp]
        lib.orc_get_velocity.argtypes = [ctypes.c_void_p, dp]
        lib.orc_total_force.argtypes = [ctypes.c_void_p, dp]
        lib.orc_diagnostics.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Diag)]
        lib.orc_lattice_tables.argtypes = [ip, ip, ip, dp, ip]
        lib.orc_feq.argtypes = [ctypes.c_double] * 4 + [dp]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
        return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice_tables():
    """(ex, ey, ez, w, opp) as the oracle defines them."""
    lib = _load()
    ex = (ctypes.c_int * 19)(); ey = (ctypes.c_int * 19)(); ez = (ctypes.c_int * 19)()
    w = (ctypes.c_double * 19)(); opp = (ctypes.c_int * 19)()
    lib.orc_lattice_tables(ex, ey, ez, w, opp)
    return (np.array(ex[:]), np.array(ey[:]), np.array(ez[:]), np.array(w[:]), np.array(opp[:]))


def num_threads() -> int:
    """Threads the oracle's per-node loops use."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int):
    """Threads of the oracle's per-node loops (results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


def feq(rho: float, u) -> np.ndarray:
    """The oracle's equilibrium f^eq_i(rho, u), Eq. (eqdis)."""
    lib = _load()
    out = np.zeros(19)
    lib.orc_feq(float(rho), float(u[0]), float(u[1]), float(u[2]), _dp(out))
    return out


@dataclasses.dataclass
class OracleParams:
    nx: int
    ny: int
    nz: int
    wall_z: bool = False
    tau: tuple = (1.0, 1.0)
    g: float = 0.9
    psi: int = PSI_RHO
    sink: int = SINK_NONE
    rho_h: float = 0.04
    sink_radius: float = 0.0
    center: tuple | None = None
    phi_delta: tuple = (0.66, -0.66)
    solid_z: int = 0
    wall_rho: tuple = (0.0, 0.0)
    ncomp: int = 2


class Oracle:
    """One lattice of the oracle. ``n = nx*ny*nz``; arrays are z-major."""

    def __init__(self, p: OracleParams):
        lib = _load()
        self.p = p
        self.shape = (p.nz, p.ny, p.nx)
        self.n = p.nx * p.ny * p.nz
        c = p.center if p.center is not None else ((p.nx - 1) / 2, (p.ny - 1) / 2, (p.nz - 1) / 2)
        cp = _Params(p.nx, p.ny, p.nz, int(p.wall_z), (ctypes.c_double * 2)(*p.tau), p.g, p.psi, p.sink,
                     p.rho_h, p.sink_radius, (ctypes.c_double * 3)(*c), (ctypes.c_double * 2)(*p.phi_delta),
                     int(p.solid_z), (ctypes.c_double * 2)(*p.wall_rho), int(p.ncomp))
        self._h = lib.orc_create(ctypes.byref(cp))
        if not self._h:
            raise ValueError("oracle: invalid lattice parameters")
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def init_from_density(self, rho_a: np.ndarray, rho_b: np.ndarray = None):
        """rho_b is ignored (may be None) for one component."""
        a = np.ascontiguousarray(rho_a, dtype=np.float64).reshape(-1)
        if rho_b is None:
            rho_b = np.zeros_like(a)
        b = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(-1)
        assert a.size == self.n and b.size == self.n
        self._lib.orc_init_from_density(self._h, _dp(a), _dp(b))

    def init_from_populations(self, f: np.ndarray):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert a.size == 2 * 19 * self.n
        self._lib.orc_init_from_populations(self._h, _dp(a))

    def set_sink(self, kind: int, rho_h: float, radius: float = 0.0):
        self._lib.orc_set_sink(self._h, kind, rho_h, radius)

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    def populations(self) -> np.ndarray:
        out = np.empty(2 * 19 * self.n)
        self._lib.orc_get_populations(self._h, _dp(out))
        return out.reshape((2, 19) + self.shape)

    def density(self):
        a = np.empty(self.n); b = np.empty(self.n)
        self._lib.orc_get_density(self._h, _dp(a), _dp(b))
        return a.reshape(self.shape), b.reshape(self.shape)

    def velocity(self) -> np.ndarray:
        out = np.empty(3 * self.n)
        self._lib.orc_get_velocity(self._h, _dp(out))
        return out.reshape((3,) + self.shape)

    def total_force(self) -> np.ndarray:
        out = np.zeros(3)
        self._lib.orc_total_force(self._h, _dp(out))
        return out

    def diagnostics(self) -> dict:
        d = _Diag()
        self._lib.orc_diagnostics(self._h, ctypes.byref(d))
        return {
            "step": d.step, "mass": (d.mass[0], d.mass[1]), "evaporated": d.evaporated,
            "evap_rate": d.evap_rate, "momentum": (d.momentum[0], d.momentum[1], d.momentum[2]),
            "z_interface": d.z_interface, "r_droplet": d.r_droplet,
            "nonfinite": d.nonfinite, "nonpositive": d.nonpositive,
        }
