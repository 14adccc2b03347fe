"""ctypes binding of libelas3d (C-ABI in include/elas3d.h).

Argument marshalling only: every step of the solve runs in the HIP kernels
of ``libelas3d.so``.  The functions keep the C names without the ``elas3d_``
prefix.  Host arrays are numpy; device arrays may be any object with a
``data_ptr()`` (torch CUDA tensors) when the context was created with
``inputs_on_device`` / ``outputs_on_device``.

There is no fallback: if the shared library is missing, importing this
module raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

__all__ = [
    "OK", "NOT_CONVERGED", "BREAKDOWN", "EBADARG", "ENOMEM", "EDEVICE", "EORDER",
    "PREC_FP64", "PREC_MIXED", "CONV_RESIDUAL", "CONV_PAPER", "PRECOND_BLOCK_JACOBI",
    "PRECOND_NONE", "TILE_SHAPES", "WS_TILES", "WS_FP32_ONLY", "Options", "Info", "Elas3dError", "lib", "LIB_PATH", "options_init",
    "setup", "solve", "stress", "apply", "get_load", "get_precond", "get_solution",
    "device_bytes", "destroy", "last_error", "version", "Context", "EXPORTS", "von_mises",
    "generate_grains", "generate_grains_static", "carve_pores", "PORE_STRIDE", "Group", "stream_bandwidth",
]

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
EBADARG, ENOMEM, EDEVICE, EORDER = -1, -2, -3, -4
PREC_FP64, PREC_MIXED = 0, 1
CONV_RESIDUAL, CONV_PAPER = 0, 1
PRECOND_BLOCK_JACOBI, PRECOND_NONE = 0, 1
MAX_RHS = 6
# workgroup shapes (compute lanes in x, y) of the direction+operator sweep, by
# options.tile; 5 and 6 add two loader wavefronts (nx a multiple of 2, of 4 in
# mixed precision; at most 96 distinct phases per workgroup box), and 6 is for
# the FP32 sweep of mixed precision only
TILE_SHAPES = ((32, 8), (16, 16), (64, 4), (32, 16), (64, 8), (64, 6), (64, 8))
WS_TILES = (5, 6)
WS_FP32_ONLY = (6,)  # wave-specialised shapes of the FP32 sweep only
# doubles per pore of elas3d_carve_pores: centre 3, semi-axes 3, R row-major 9
PORE_STRIDE = 15

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libelas3d.so")

EXPORTS = (
    "elas3d_options_init", "elas3d_setup", "elas3d_solve", "elas3d_stress", "elas3d_apply",
    "elas3d_get_load", "elas3d_get_precond", "elas3d_get_solution", "elas3d_device_bytes",
    "elas3d_destroy", "elas3d_last_error", "elas3d_version", "elas3d_von_mises",
    "elas3d_generate_grains", "elas3d_carve_pores", "elas3d_group_create", "elas3d_group_add",
    "elas3d_group_run", "elas3d_group_destroy", "elas3d_stream_bandwidth", "elas3d_generate_grains_static",
)


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("convergence", ctypes.c_int32),
        ("preconditioner", ctypes.c_int32),
        ("inputs_on_device", ctypes.c_int32),
        ("outputs_on_device", ctypes.c_int32),
        ("poll_interval", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("inner_tol", ctypes.c_double),
        ("inner_maxit", ctypes.c_int32),
        ("batched", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("zchunk", ctypes.c_int32),
        ("update_blocks", ctypes.c_int32),
        ("update_nontemporal", ctypes.c_int32),
    ]


_R = MAX_RHS


class Info(ctypes.Structure):
    _fields_ = [
        ("nrhs", ctypes.c_int32),
        ("status", ctypes.c_int32 * _R),
        ("iters", ctypes.c_int32 * _R),
        ("restarts", ctypes.c_int32 * _R),
        ("relres_true", ctypes.c_double * _R),
        ("relres_recursive", ctypes.c_double * _R),
        ("relres_precond", ctypes.c_double * _R),
        ("t_solve_s", ctypes.c_double),
        ("bytes_per_iter", ctypes.c_double),
        ("t_operator_ms", ctypes.c_double),
        ("n_operator", ctypes.c_int64),
        ("t_update_ms", ctypes.c_double),
        ("n_update", ctypes.c_int64),
        ("fp64_fallback", ctypes.c_int32 * _R),
        ("op_tile", ctypes.c_int32 * 3),
        ("update_blocks", ctypes.c_int32),
        ("precond_rows", ctypes.c_int64),
        ("update_nontemporal", ctypes.c_int32),
        ("apply_tile", ctypes.c_int32 * 3),
        ("op_shape", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        n = self.nrhs
        return {
            "nrhs": n,
            "status": list(self.status[:n]),
            "iters": list(self.iters[:n]),
            "restarts": list(self.restarts[:n]),
            "relres_true": list(self.relres_true[:n]),
            "relres_recursive": list(self.relres_recursive[:n]),
            "relres_precond": list(self.relres_precond[:n]),
            "t_solve_s": self.t_solve_s,
            "bytes_per_iter": self.bytes_per_iter,
            "t_operator_ms": self.t_operator_ms,
            "n_operator": self.n_operator,
            "t_update_ms": self.t_update_ms,
            "n_update": self.n_update,
            "fp64_fallback": list(self.fp64_fallback[:n]),
            "op_tile": list(self.op_tile),
            "update_blocks": self.update_blocks,
            "precond_rows": self.precond_rows,
            "update_nontemporal": self.update_nontemporal,
            "apply_tile": list(self.apply_tile),
            "op_shape": self.op_shape,
        }


class Elas3dError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"elas3d error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libelas3d.so (raises if it has not been built).

    PyTorch wheels carry their own HIP runtime with the same soname as the
    system one.  torch is imported first, when installed, so that the
    library binds to that runtime: one HIP runtime per process, and torch's
    device pointers and streams are valid in the library's calls.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_2602_07354_amd.build")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.elas3d_options_init.argtypes = [ctypes.POINTER(Options)]
        L.elas3d_options_init.restype = None
        L.elas3d_setup.argtypes = [ctypes.POINTER(vp), i32, i32, i32, vp, i32, vp, i32, vp,
                                   ctypes.POINTER(Options)]
        L.elas3d_setup.restype = ctypes.c_int
        L.elas3d_solve.argtypes = [vp, d, i32, i32, ctypes.POINTER(Info)]
        L.elas3d_solve.restype = ctypes.c_int
        L.elas3d_stress.argtypes = [vp, i32, vp, vp, vp, vp]
        L.elas3d_stress.restype = ctypes.c_int
        L.elas3d_apply.argtypes = [vp, vp, vp]
        L.elas3d_apply.restype = ctypes.c_int
        L.elas3d_get_load.argtypes = [vp, i32, vp]
        L.elas3d_get_load.restype = ctypes.c_int
        L.elas3d_get_precond.argtypes = [vp, vp]
        L.elas3d_get_precond.restype = ctypes.c_int
        L.elas3d_get_solution.argtypes = [vp, i32, vp]
        L.elas3d_get_solution.restype = ctypes.c_int
        L.elas3d_device_bytes.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(Options)]
        L.elas3d_device_bytes.restype = ctypes.c_double
        L.elas3d_destroy.argtypes = [vp]
        L.elas3d_destroy.restype = None
        L.elas3d_last_error.argtypes = [vp]
        L.elas3d_last_error.restype = ctypes.c_char_p
        L.elas3d_version.argtypes = []
        L.elas3d_version.restype = ctypes.c_char_p
        L.elas3d_von_mises.argtypes = [vp, i32, vp, vp, vp]
        L.elas3d_von_mises.restype = ctypes.c_int
        L.elas3d_generate_grains.argtypes = [i32, i32, i32, i32, vp, vp, vp, ctypes.POINTER(Options)]
        L.elas3d_generate_grains.restype = ctypes.c_int
        L.elas3d_generate_grains_static.argtypes = [i32, i32, i32, i32, vp, vp, vp, ctypes.POINTER(Options)]
        L.elas3d_generate_grains_static.restype = ctypes.c_int
        L.elas3d_carve_pores.argtypes = [i32, i32, i32, vp, i32, i32, vp, d, vp, vp,
                                         ctypes.POINTER(Options)]
        L.elas3d_carve_pores.restype = ctypes.c_int
        L.elas3d_group_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Options)]
        L.elas3d_group_create.restype = ctypes.c_int
        L.elas3d_group_add.argtypes = [vp, vp, d, i32]
        L.elas3d_group_add.restype = ctypes.c_int
        L.elas3d_group_run.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(Info), i32,
                                       ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.elas3d_group_run.restype = ctypes.c_int
        L.elas3d_group_destroy.argtypes = [vp]
        L.elas3d_group_destroy.restype = None
        L.elas3d_stream_bandwidth.argtypes = [ctypes.c_int64, i32, i32, i32, vp, ctypes.POINTER(Options)]
        L.elas3d_stream_bandwidth.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a) -> Optional[int]:
    """Address of a numpy array (host) or of an object with data_ptr() (device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        return int(a.data_ptr())
    if isinstance(a, int):
        return a
    raise TypeError(f"cannot pass {type(a)} to the C-ABI")


def options_init(**kw) -> Options:
    o = Options()
    lib().elas3d_options_init(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def last_error(ctx=None) -> str:
    return lib().elas3d_last_error(ctx).decode()


def version() -> str:
    return lib().elas3d_version().decode()


def _check(rc: int, ctx=None, soft_ok: bool = False) -> int:
    if rc < 0 or (rc > 0 and not soft_ok):
        raise Elas3dError(rc, last_error(ctx))
    return rc


def setup(shape, phase, C, strain, options: Optional[Options] = None):
    """elas3d_setup; returns an opaque context handle (int)."""
    nx, ny, nz = (int(s) for s in shape)
    C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1, 36)
    strain = np.ascontiguousarray(strain, dtype=np.float64).reshape(-1, 6)
    if isinstance(phase, np.ndarray):
        phase = np.ascontiguousarray(phase, dtype=np.int32)
    h = ctypes.c_void_p()
    rc = lib().elas3d_setup(ctypes.byref(h), nx, ny, nz, _ptr(phase), C.shape[0], _ptr(C),
                            strain.shape[0], _ptr(strain),
                            ctypes.byref(options) if options is not None else None)
    _check(rc)
    return h.value


def solve(ctx, tol: float, maxit: int, nrhs: int = 1) -> tuple:
    """elas3d_solve; returns (status, Info)."""
    info = Info()
    rc = lib().elas3d_solve(ctx, float(tol), int(maxit), int(nrhs), ctypes.byref(info))
    _check(rc, ctx, soft_ok=True)
    return rc, info


def stress(ctx, rhs: int, sigma_voxel=None, sigma_avg=None, u_node=None, energy=None) -> int:
    return _check(lib().elas3d_stress(ctx, int(rhs), _ptr(sigma_voxel), _ptr(sigma_avg),
                                      _ptr(u_node), _ptr(energy)), ctx)


def apply(ctx, x, y) -> int:
    return _check(lib().elas3d_apply(ctx, _ptr(x), _ptr(y)), ctx)


def get_load(ctx, rhs: int, b) -> int:
    return _check(lib().elas3d_get_load(ctx, int(rhs), _ptr(b)), ctx)


def get_precond(ctx, minv) -> int:
    return _check(lib().elas3d_get_precond(ctx, _ptr(minv)), ctx)


def get_solution(ctx, rhs: int, w) -> int:
    return _check(lib().elas3d_get_solution(ctx, int(rhs), _ptr(w)), ctx)


def von_mises(ctx, rhs: int, vm=None) -> tuple:
    """elas3d_von_mises; fills vm (N doubles or None), returns (max, argmax)."""
    mx = np.empty(1)
    am = np.empty(1, dtype=np.int64)
    _check(lib().elas3d_von_mises(ctx, int(rhs), _ptr(vm), _ptr(mx), _ptr(am)), ctx)
    return float(mx[0]), int(am[0])


def generate_grains(shape, seeds, semi=None, phase=None, options: Optional[Options] = None):
    """elas3d_generate_grains.  Host phase (returned) unless options has
    outputs_on_device and `phase` is a device buffer of N int32."""
    nx, ny, nz = (int(s) for s in shape)
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    if semi is not None:
        semi = np.ascontiguousarray(semi, dtype=np.float64).reshape(-1, 2)
        if semi.shape[0] != seeds.shape[0]:
            raise ValueError("semi must have one row per seed")
    if phase is None:
        phase = np.empty(nx * ny * nz, dtype=np.int32)
    rc = lib().elas3d_generate_grains(nx, ny, nz, seeds.shape[0], _ptr(seeds), _ptr(semi), _ptr(phase),
                                      ctypes.byref(options) if options is not None else None)
    _check(rc)
    return phase


def generate_grains_static(shape, seeds, semi, phase, options: Options):
    """elas3d_generate_grains_static: the allocation-free grain assignment into
    the device buffer `phase` (options.outputs_on_device must be set)."""
    nx, ny, nz = (int(s) for s in shape)
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    if semi is not None:
        semi = np.ascontiguousarray(semi, dtype=np.float64).reshape(-1, 2)
        if semi.shape[0] != seeds.shape[0]:
            raise ValueError("semi must have one row per seed")
    rc = lib().elas3d_generate_grains_static(nx, ny, nz, seeds.shape[0], _ptr(seeds), _ptr(semi), _ptr(phase),
                                             ctypes.byref(options) if options is not None else None)
    _check(rc)
    return phase


def carve_pores(shape, phase, void_id: int, pores, target: float = -1.0,
                options: Optional[Options] = None) -> tuple:
    """elas3d_carve_pores on `phase` in place; returns (pores used, void voxels)."""
    nx, ny, nz = (int(s) for s in shape)
    pores = np.ascontiguousarray(pores, dtype=np.float64).reshape(-1, PORE_STRIDE)
    used = np.zeros(1, dtype=np.int32)
    nvoid = np.zeros(1, dtype=np.int64)
    rc = lib().elas3d_carve_pores(nx, ny, nz, _ptr(phase), int(void_id), pores.shape[0],
                                  _ptr(pores) if pores.shape[0] else None, float(target), _ptr(used),
                                  _ptr(nvoid), ctypes.byref(options) if options is not None else None)
    _check(rc)
    return int(used[0]), int(nvoid[0])


def device_bytes(shape, nphase: int, nrhs: int, options: Optional[Options] = None) -> float:
    nx, ny, nz = (int(s) for s in shape)
    return lib().elas3d_device_bytes(nx, ny, nz, int(nphase), int(nrhs),
                                     ctypes.byref(options) if options is not None else None)


def stream_bandwidth(nbytes: int, blocks: int = 32768, reps: int = 5, nontemporal: bool = False,
                     options: Optional[Options] = None) -> dict:
    """elas3d_stream_bandwidth: copy, read and write rates in GB/s (1e9 B/s)."""
    gbs = np.zeros(3)
    rc = lib().elas3d_stream_bandwidth(int(nbytes), int(blocks), int(reps), int(bool(nontemporal)),
                                       _ptr(gbs), ctypes.byref(options) if options is not None else None)
    _check(rc)
    return {"copy": float(gbs[0]), "read": float(gbs[1]), "write": float(gbs[2])}


def destroy(ctx) -> None:
    if ctx:
        lib().elas3d_destroy(ctx)


class Context:
    """Owning wrapper of one elas3d context (host numpy in/out by default)."""

    def __init__(self, shape, phase, C, strain, **opts):
        self.shape = tuple(int(s) for s in shape)
        self.n = int(np.prod(self.shape))
        self.nrhs = int(np.asarray(strain).reshape(-1, 6).shape[0])
        self.options = options_init(**opts)
        self.handle = setup(self.shape, phase, C, strain, self.options)

    @classmethod
    def from_micro(cls, ms, **opts):
        return cls(ms.shape, ms.phase, ms.C, ms.strain, **opts)

    def solve(self, tol: float, maxit: int = 100000, nrhs: Optional[int] = None):
        st, info = solve(self.handle, tol, maxit, self.nrhs if nrhs is None else nrhs)
        return st, info.as_dict()

    def stress(self, rhs: int = 0, voxel: bool = True, displacement: bool = False) -> dict:
        sig = np.empty((6, self.n)) if voxel else None
        avg = np.empty(6)
        u = np.empty((3, self.n)) if displacement else None
        en = np.empty(1)
        stress(self.handle, rhs, sig, avg, u, en)
        return {"sigma": sig, "avg": avg, "u": u, "energy": float(en[0])}

    def apply(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(3, self.n)
        y = np.empty_like(x)
        apply(self.handle, x, y)
        return y

    def load(self, rhs: int = 0) -> np.ndarray:
        b = np.empty((3, self.n))
        get_load(self.handle, rhs, b)
        return b

    def precond(self) -> np.ndarray:
        """(N, 3, 3) symmetric inverse blocks from the six stored planes."""
        m = np.empty((6, self.n))
        get_precond(self.handle, m)
        out = np.empty((self.n, 3, 3))
        xx, yy, zz, yz, xz, xy = m
        out[:, 0, 0], out[:, 1, 1], out[:, 2, 2] = xx, yy, zz
        out[:, 1, 2] = out[:, 2, 1] = yz
        out[:, 0, 2] = out[:, 2, 0] = xz
        out[:, 0, 1] = out[:, 1, 0] = xy
        return out

    def von_mises(self, rhs: int = 0, field: bool = True) -> dict:
        vm = np.empty(self.n) if field else None
        mx, am = von_mises(self.handle, rhs, vm)
        return {"vm": vm, "max": mx, "argmax": am}

    def solution(self, rhs: int = 0) -> np.ndarray:
        w = np.empty((3, self.n))
        get_solution(self.handle, rhs, w)
        return w

    def close(self):
        if self.handle:
            destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Continuous batching of independent solves (elas3d_group_*): members
    advance in lockstep with one launch per sweep for all of them."""

    def __init__(self, options: Optional[Options] = None):
        h = ctypes.c_void_p()
        _check(lib().elas3d_group_create(ctypes.byref(h), ctypes.byref(options) if options is not None else None))
        self.handle = h.value

    def add(self, ctx, tol: float, maxit: int = 100000) -> None:
        """Admit a context handle (all its load cases)."""
        _check(lib().elas3d_group_add(self.handle, ctx, float(tol), int(maxit)))

    def run(self, iters: int, cap: int = 64) -> tuple:
        """Run `iters` lockstep iterations; returns ([(ctx, status, info dict)], active)."""
        done = (ctypes.c_void_p * max(cap, 1))()
        infos = (Info * max(cap, 1))()
        nd, na = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().elas3d_group_run(self.handle, int(iters), done, infos, int(cap), ctypes.byref(nd),
                                      ctypes.byref(na)))
        out = []
        for k in range(nd.value):
            info = infos[k].as_dict()
            out.append((done[k], max(info["status"]), info))
        return out, na.value

    def close(self):
        if self.handle:
            lib().elas3d_group_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
