"""ctypes wrapper around the plain-C FP64 oracle (el_oracle.c).

TEST INFRASTRUCTURE ONLY.  Arrays cross the interface as float64 numpy arrays
in the external layout field[c][zf][y][x] over fluid layers (see el_oracle.h).
Citations of the paper are in el_oracle.c next to each equation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "el_oracle.c")
_LIB = os.path.join(_HERE, "libel_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction of a*b+c into fma)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic_z", C.c_int32), ("shifted", C.c_int32), ("fd_ratio", C.c_int32),
                ("renorm_predictor", C.c_int32), ("coupling", C.c_int32),
                ("tau", C.c_double), ("g", C.c_double * 3),
                ("K", C.c_double), ("q0", C.c_double), ("W0", C.c_double),
                ("alpha", C.c_double * 6), ("alpha4p", C.c_double),
                ("frank3", C.c_int32), ("free_walls", C.c_int32),
                ("K11", C.c_double), ("K22", C.c_double), ("K33", C.c_double)]


class _Obs(C.Structure):
    _fields_ = [("mass", C.c_double), ("mom", C.c_double * 3), ("mom_phys", C.c_double * 3),
                ("max_u", C.c_double), ("max_unit_dev", C.c_double), ("nonfinite", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def load_library(path: str):
    """Load an oracle shared library at `path` and declare its functions."""
    lib = C.CDLL(path)
    D = C.POINTER(C.c_double)
    lib.or_create.restype = C.c_void_p
    lib.or_create.argtypes = [C.POINTER(_Params)]
    lib.or_destroy.argtypes = [C.c_void_p]
    lib.or_set_threads.argtypes = [C.c_int32]
    lib.or_init.argtypes = [C.c_void_p, D]
    lib.or_init_flow.argtypes = [C.c_void_p, D]
    lib.or_step_lbm.argtypes = [C.c_void_p, C.c_int32]
    lib.or_step_director.argtypes = [C.c_void_p]
    lib.or_run.argtypes = [C.c_void_p, C.c_int64]
    lib.or_step_count.restype = C.c_int64
    lib.or_step_count.argtypes = [C.c_void_p]
    lib.or_get.argtypes = [C.c_void_p, C.c_int32, D]
    lib.or_set.argtypes = [C.c_void_p, C.c_int32, D]
    lib.or_moments.argtypes = [C.c_void_p]
    lib.or_force.argtypes = [C.c_void_p]
    lib.or_molecular_field.argtypes = [C.c_void_p, D]
    lib.or_director_rhs.argtypes = [C.c_void_p, D, D]
    lib.or_stress.argtypes = [C.c_void_p, C.c_int32, D]
    lib.or_force_masked.argtypes = [C.c_void_p, C.c_int32, D]
    lib.or_observables.argtypes = [C.c_void_p, C.POINTER(_Obs)]
    lib.or_tube_centroids.argtypes = [C.c_void_p, C.c_int32, D, D, D]
    lib.or_set_obstacles.argtypes = [C.c_void_p, C.c_void_p]
    lib.or_lattice.argtypes = [D, D, C.POINTER(C.c_int32)]
    lib.or_equilibrium.argtypes = [C.c_double, C.c_double, D, C.c_int32, D]
    lib.or_guo_source.argtypes = [D, D, D]
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lattice():
    """Return (e[19,3], w[19], opp[19]) of the oracle's D3Q19 set."""
    lib = _load()
    e = np.zeros((19, 3))
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib.or_lattice(_dp(e), _dp(w), opp.ctypes.data_as(C.POINTER(C.c_int32)))
    return e, w, opp


def equilibrium(rho: float, u, shifted: bool) -> np.ndarray:
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib.or_equilibrium(float(rho), float(rho) - 1.0, _dp(uu), int(shifted), _dp(out))
    return out


def guo_source(u, F) -> np.ndarray:
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64)
    ff = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib.or_guo_source(_dp(uu), _dp(ff), _dp(out))
    return out


@dataclass
class OracleParams:
    nx: int
    ny: int
    nz: int
    tau: float = 0.8
    g: tuple = (0.0, 0.0, 0.0)
    K: float = 0.0
    q0: float = 0.0
    W0: float = 0.0
    alpha: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    alpha4p: float = 0.0
    fd_ratio: int = 1
    shifted: bool = True
    periodic_z: bool = False
    renorm_predictor: bool = True
    coupling: bool = True
    frank3: bool = False
    free_walls: bool = False
    K11: float = 0.0
    K22: float = 0.0
    K33: float = 0.0

    @property
    def nzf(self) -> int:
        return self.nz if self.periodic_z else self.nz - 2

    def to_c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.periodic_z = int(self.periodic_z)
        p.shifted = int(self.shifted)
        p.fd_ratio = int(self.fd_ratio)
        p.renorm_predictor = int(self.renorm_predictor)
        p.coupling = int(self.coupling)
        p.tau = self.tau
        p.g = (C.c_double * 3)(*self.g)
        p.K, p.q0, p.W0 = self.K, self.q0, self.W0
        p.alpha = (C.c_double * 6)(*self.alpha)
        p.alpha4p = self.alpha4p
        p.frank3 = int(self.frank3)
        p.free_walls = int(self.free_walls)
        p.K11, p.K22, p.K33 = self.K11, self.K22, self.K33
        return p


_NCOMP = {0: 19, 1: 3, 2: 3, 3: 3, 4: 3}
_WHICH = {"q": 0, "n": 1, "nP": 2, "u": 3, "F": 4}


class Oracle:
    """One oracle lattice; fields in external layout, shape (c, nzf, ny, nx)."""

    def __init__(self, params: OracleParams, threads: int = 1):
        self.p = params
        self.lib = _load()
        self.lib.or_set_threads(int(threads))
        self._cp = params.to_c()
        self.h = self.lib.or_create(C.byref(self._cp))

    def close(self):
        if self.h:
            self.lib.or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_threads(self, threads: int):
        self.lib.or_set_threads(int(threads))

    @property
    def shape(self):
        return (self.p.nzf, self.p.ny, self.p.nx)

    def _arr(self, ncomp):
        return np.zeros((ncomp,) + self.shape)

    def set_obstacles(self, mask):
        """Solid nodes inside the channel: a (nzf, ny, nx) mask (nonzero =
        solid), or None.  Call before init()."""
        if mask is None:
            self.lib.or_set_obstacles(self.h, None)
            return
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8).reshape(self.shape)
        self._mask = m
        self.lib.or_set_obstacles(self.h, m.ctypes.data_as(C.c_void_p))

    def init(self, n0: np.ndarray):
        a = np.ascontiguousarray(n0, dtype=np.float64).reshape((3,) + self.shape)
        self.lib.or_init(self.h, _dp(a))

    def init_flow(self, u0: np.ndarray):
        a = np.ascontiguousarray(u0, dtype=np.float64).reshape((3,) + self.shape)
        self.lib.or_init_flow(self.h, _dp(a))

    def step_lbm(self, nsteps: int = 1):
        self.lib.or_step_lbm(self.h, int(nsteps))

    def step_director(self):
        self.lib.or_step_director(self.h)

    def run(self, T: int):
        self.lib.or_run(self.h, int(T))

    @property
    def t(self) -> int:
        return int(self.lib.or_step_count(self.h))

    def get(self, name: str) -> np.ndarray:
        w = _WHICH[name]
        out = self._arr(_NCOMP[w])
        self.lib.or_get(self.h, w, _dp(out))
        return out

    def set(self, name: str, arr: np.ndarray):
        w = _WHICH[name]
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape((_NCOMP[w],) + self.shape)
        self.lib.or_set(self.h, w, _dp(a))

    def moments(self):
        self.lib.or_moments(self.h)

    def force(self):
        self.lib.or_force(self.h)

    def molecular_field(self) -> np.ndarray:
        out = self._arr(3)
        self.lib.or_molecular_field(self.h, _dp(out))
        return out

    def director_rhs(self, m: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(m, dtype=np.float64).reshape((3,) + self.shape)
        out = self._arr(3)
        self.lib.or_director_rhs(self.h, _dp(a), _dp(out))
        return out

    def stress(self, term_mask: int = 127) -> np.ndarray:
        out = self._arr(9)
        self.lib.or_stress(self.h, int(term_mask), _dp(out))
        return out.reshape((3, 3) + self.shape)

    def force_masked(self, term_mask: int = 127) -> np.ndarray:
        out = self._arr(3)
        self.lib.or_force_masked(self.h, int(term_mask), _dp(out))
        return out

    def observables(self) -> dict:
        o = _Obs()
        self.lib.or_observables(self.h, C.byref(o))
        return {"mass": o.mass, "mom": np.array(o.mom[:]), "mom_phys": np.array(o.mom_phys[:]),
                "max_u": o.max_u, "max_unit_dev": o.max_unit_dev, "nonfinite": int(o.nonfinite)}

    def tube_centroids(self, seeds):
        """Per-tube weight sums and circular-mean centroids of the stored director
        for tube seeds [(x, y), ...] (at most 64)."""
        sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.float64).reshape(-1, 2))
        nt = sd.shape[0]
        assert 1 <= nt <= 64
        w = np.zeros(nt)
        c = np.zeros((nt, 2))
        self.lib.or_tube_centroids(self.h, nt, _dp(sd), _dp(w), _dp(c))
        return w, c
