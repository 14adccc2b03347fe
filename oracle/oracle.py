"""ctypes wrapper of the C oracle (test infrastructure only; see package doc)."""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

__all__ = [
    "build", "lib", "Problem", "element_stiffness", "stiffness_table",
    "CONVERGED", "NOT_CONVERGED", "BREAKDOWN", "grains", "grains_at", "carve", "covered_at", "von_mises",
    "threaded_available",
]

CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "elas3d_oracle.c")
_SRC_GEN = os.path.join(_HERE, "microstructure_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same sources built with OpenMP: only for timing a threaded CPU baseline
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _stale(path: str = _LIB) -> bool:
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    return any(t < os.path.getmtime(src) for src in (_SRC, _SRC_GEN))


def _compile(path: str, extra) -> None:
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", *extra, "-o", tmp,
                           _SRC, _SRC_GEN, "-lm"])
    os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction),
    and the OpenMP build of the same sources used to time the threaded CPU
    baseline (skipped quietly when the compiler has no OpenMP)."""
    if force or _stale():
        _compile(_LIB, [])
    if force or _stale(_LIB_OMP):
        try:
            _compile(_LIB_OMP, ["-fopenmp"])
        except (subprocess.CalledProcessError, OSError):
            pass
    return _LIB


def threaded_available() -> bool:
    """True when the OpenMP build of the oracle is present (or can be built)."""
    if _stale(_LIB_OMP):
        try:
            _compile(_LIB_OMP, ["-fopenmp"])
        except (subprocess.CalledProcessError, OSError):
            return False
    return os.path.exists(_LIB_OMP)


def _declare(L):
    i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
    L.orc_element_stiffness.argtypes = [_D, _D]
    L.orc_stiffness_table.argtypes = [i, _D, _D]
    L.orc_apply.argtypes = [i, i, i, _I32, _D, _D, _D]
    L.orc_apply_at.argtypes = [i, i, i, _I32, _D, _D, _I64, l, _D]
    L.orc_load.argtypes = [i, i, i, _I32, _D, _D, _D, _D]
    L.orc_load_at.argtypes = [i, i, i, _I32, _D, _D, _I64, l, _D]
    L.orc_precond.argtypes = [i, i, i, _I32, _D, i, _D, i, _D]
    L.orc_precond_at.argtypes = [i, i, i, _I32, _D, i, _D, _I64, l, _D]
    L.orc_pcg.argtypes = [i, i, i, _I32, _D, _D, _D, d, d, i, i, _D, _D, _D]
    L.orc_pcg.restype = ctypes.c_int
    L.orc_stress.argtypes = [i, i, i, _I32, i, _D, _D, _D, _D, _D]
    L.orc_energy.argtypes = [i, i, i, _I32, _D, _D, _D]
    L.orc_energy.restype = d
    L.orc_grains.argtypes = [i, i, i, i, _D, _D, _I32]
    L.orc_carve.argtypes = [i, i, i, _I32, ctypes.c_int32, i, _D, d, _I64]
    L.orc_carve.restype = ctypes.c_int
    L.orc_von_mises.argtypes = [l, _D, _D]
    L.orc_grains_at.argtypes = [i, i, i, i, _D, _D, _I64, l, _I32]
    L.orc_covered_at.argtypes = [i, i, i, i, _D, _I64, l, _I32]
    L.orc_set_threads.argtypes = [i]
    return L


def threaded_lib(threads: int):
    """The OpenMP build, set to `threads` threads (timing only)."""
    global _lib_omp
    if _lib_omp is None:
        if not threaded_available():
            raise RuntimeError("the OpenMP build of the oracle is not available")
        _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
    _lib_omp.orc_set_threads(int(threads))
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _p(a, t=_D):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def element_stiffness(C: np.ndarray) -> np.ndarray:
    """24x24 K_e of the unit voxel for a 6x6 Voigt stiffness (dof 3*a + c)."""
    C = _f64(C).reshape(36)
    ke = np.empty(576)
    lib().orc_element_stiffness(_p(C), _p(ke))
    return ke.reshape(24, 24)


def stiffness_table(C: np.ndarray) -> np.ndarray:
    C = _f64(C).reshape(-1, 36)
    ke = np.empty((C.shape[0], 576))
    lib().orc_stiffness_table(C.shape[0], _p(C), _p(ke))
    return ke


class Problem:
    """One microstructure: grid, phase map and per-phase stiffness."""

    def __init__(self, shape, phase, C, threads: int = 0):
        """threads > 0 runs the OpenMP build on that many threads (timing
        only; its sums are formed in another order)."""
        self._L = lib() if threads <= 0 else threaded_lib(threads)
        self.nx, self.ny, self.nz = (int(s) for s in shape)
        self.n = self.nx * self.ny * self.nz
        self.phase = np.ascontiguousarray(phase, dtype=np.int32).reshape(self.n)
        self.C = _f64(C).reshape(-1, 6, 6)
        self.nphase = self.C.shape[0]
        self.ke = stiffness_table(self.C)

    @classmethod
    def from_micro(cls, ms):
        return cls(ms.shape, ms.phase, ms.C)

    def _g(self):
        return self.nx, self.ny, self.nz

    def apply(self, x: np.ndarray) -> np.ndarray:
        x = _f64(x).reshape(3, self.n)
        y = np.empty_like(x)
        self._L.orc_apply(*self._g(), _p(self.phase, _I32), _p(self.ke), _p(x), _p(y))
        return y

    def apply_at(self, x: np.ndarray, nodes: np.ndarray) -> np.ndarray:
        x = _f64(x).reshape(3, self.n)
        sel = np.ascontiguousarray(nodes, dtype=np.int64)
        y = np.empty((3, sel.size))
        self._L.orc_apply_at(*self._g(), _p(self.phase, _I32), _p(self.ke), _p(x),
                           _p(sel, _I64), sel.size, _p(y))
        return y

    def load(self, strain) -> tuple:
        """(b, ||b||_ref^2) for one macroscopic strain (tensor components)."""
        e = _f64(strain).reshape(6)
        b = np.empty((3, self.n))
        r2 = np.zeros(1)
        self._L.orc_load(*self._g(), _p(self.phase, _I32), _p(self.ke), _p(e), _p(b), _p(r2))
        return b, float(r2[0])

    def load_at(self, strain, nodes) -> np.ndarray:
        e = _f64(strain).reshape(6)
        sel = np.ascontiguousarray(nodes, dtype=np.int64)
        b = np.empty((3, sel.size))
        self._L.orc_load_at(*self._g(), _p(self.phase, _I32), _p(self.ke), _p(e),
                          _p(sel, _I64), sel.size, _p(b))
        return b

    def precond(self, identity: bool = False) -> np.ndarray:
        """N x 3 x 3 inverse diagonal blocks (0 on void-only nodes)."""
        minv = np.empty((self.n, 9))
        self._L.orc_precond(*self._g(), _p(self.phase, _I32), _p(self.ke), self.nphase,
                          _p(self.C), int(identity), _p(minv))
        return minv.reshape(self.n, 3, 3)

    def precond_at(self, nodes) -> np.ndarray:
        sel = np.ascontiguousarray(nodes, dtype=np.int64)
        minv = np.empty((sel.size, 9))
        self._L.orc_precond_at(*self._g(), _p(self.phase, _I32), _p(self.ke), self.nphase,
                             _p(self.C), _p(sel, _I64), sel.size, _p(minv))
        return minv.reshape(sel.size, 3, 3)

    def solve(self, strain, tol: float = 1e-10, maxit: int = 100000, mode: int = 0,
              preconditioned: bool = True, b: Optional[np.ndarray] = None,
              minv: Optional[np.ndarray] = None, trace: bool = False) -> dict:
        """PCG (Algorithm 2) or plain CG from w = 0; returns w and statistics."""
        if b is None:
            b, r2 = self.load(strain)
        else:
            r2 = float(np.sum(_f64(b) ** 2))
        if minv is None:
            minv = self.precond(identity=not preconditioned)
        b = _f64(b).reshape(3, self.n)
        minv = _f64(minv).reshape(self.n, 9)
        w = np.empty((3, self.n))
        info = np.zeros(5)
        tr = np.zeros(max(1, maxit)) if trace else None
        st = self._L.orc_pcg(*self._g(), _p(self.phase, _I32), _p(self.ke), _p(minv), _p(b),
                           r2, float(tol), int(maxit), int(mode), _p(w), _p(info),
                           _p(tr) if trace else None)
        out = {"w": w, "status": int(st), "iters": int(info[0]), "relres": info[1],
               "relres_precond": info[2], "relres_true": info[3], "restarts": int(info[4]),
               "b": b}
        if trace:
            out["trace"] = tr[: int(info[0])]
        return out

    def stress(self, strain, w) -> tuple:
        """(sigma 6 x N, mean stress 6) at voxel centroids."""
        e = _f64(strain).reshape(6)
        w = _f64(w).reshape(3, self.n)
        sig = np.empty((6, self.n))
        avg = np.empty(6)
        self._L.orc_stress(*self._g(), _p(self.phase, _I32), self.nphase, _p(self.C), _p(e),
                         _p(w), _p(sig), _p(avg))
        return sig, avg

    def energy(self, strain, w) -> float:
        e = _f64(strain).reshape(6)
        w = _f64(w).reshape(3, self.n)
        return float(self._L.orc_energy(*self._g(), _p(self.phase, _I32), _p(self.ke), _p(e), _p(w)))


# ------------------------------------------------------------ generator


def grains(shape, seeds, semi=None) -> np.ndarray:
    """Grain id per voxel: smallest ellipsoidal distance over all grains
    (Sec. 2.2.2, Eq. ellipsoid_dist), brute force."""
    nx, ny, nz = (int(s) for s in shape)
    seeds = _f64(seeds).reshape(-1, 3)
    semi = np.ones((seeds.shape[0], 2)) if semi is None else _f64(semi).reshape(-1, 2)
    out = np.empty(nx * ny * nz, dtype=np.int32)
    lib().orc_grains(nx, ny, nz, seeds.shape[0], _p(seeds), _p(semi), _p(out, _I32))
    return out


def grains_at(shape, seeds, semi, idx) -> np.ndarray:
    """grains() at the voxels idx only."""
    nx, ny, nz = (int(s) for s in shape)
    seeds = _f64(seeds).reshape(-1, 3)
    semi = np.ones((seeds.shape[0], 2)) if semi is None else _f64(semi).reshape(-1, 2)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.int32)
    lib().orc_grains_at(nx, ny, nz, seeds.shape[0], _p(seeds), _p(semi), _p(idx, _I64), idx.size,
                        _p(out, _I32))
    return out


def covered_at(shape, pores, idx) -> np.ndarray:
    """1 where any of the pores covers voxel idx[t] (the pore-overwrite test)."""
    nx, ny, nz = (int(s) for s in shape)
    pores = _f64(pores).reshape(-1, 15)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.int32)
    lib().orc_covered_at(nx, ny, nz, pores.shape[0], _p(pores), _p(idx, _I64), idx.size, _p(out, _I32))
    return out


def carve(shape, phase, void_id: int, pores, target: float = -1.0) -> tuple:
    """Pore overwrite in order until the void count reaches target (Sec. 2.2.3);
    returns (new phase, pores used, void voxels)."""
    nx, ny, nz = (int(s) for s in shape)
    ph = np.array(phase, dtype=np.int32, copy=True)
    pores = _f64(pores).reshape(-1, 15)
    nvoid = np.zeros(1, dtype=np.int64)
    used = lib().orc_carve(nx, ny, nz, _p(ph, _I32), int(void_id), pores.shape[0], _p(pores), float(target),
                           _p(nvoid, _I64))
    return ph, int(used), int(nvoid[0])


def von_mises(sigma) -> np.ndarray:
    """Von Mises equivalent stress of Voigt stress planes (6 x N)."""
    sigma = _f64(sigma).reshape(6, -1)
    vm = np.empty(sigma.shape[1])
    lib().orc_von_mises(sigma.shape[1], _p(sigma), _p(vm))
    return vm
