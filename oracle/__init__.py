"""CPU oracle for the SGM hot path (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path (the HIP library and its
binding) never does, and shares no code with it.

The arithmetic lives in ``sgm_oracle.c`` (plain loops, compiled with gcc);
this module marshals numpy arrays to it.  Each function names the passage
of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgm_oracle.c")
_LIB = os.path.join(_HERE, "libsgm_oracle.so")

# path index -> direction r = (du, dv); the predecessor of p is p - r
PATHS = [(+1, 0), (-1, 0), (0, +1), (0, -1), (+1, +1), (-1, +1), (+1, -1), (-1, -1)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over path directions)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.oracle_census.argtypes = [P, I, I, I, I, P]
        lib.oracle_cost.argtypes = [P, P, I, I, I, I, P, P]
        lib.oracle_path.argtypes = [P, I, I, I, I, I, I, I, P]
        lib.oracle_path_raw.argtypes = [P, I, I, I, I, I, I, I, P]
        lib.oracle_sum.argtypes = [P, I, I, I, I, I, I, P]
        lib.oracle_wta.argtypes = [P, I, I, I, P, P, P]
        lib.oracle_sgm.argtypes = [P, P, I, I, I, I, I, I, I, I, P, P, P]
        lib.oracle_window_from_road.argtypes = [D, D, D, I, I, I, I, D, P]
        lib.oracle_num_threads.argtypes = []
        lib.oracle_set_num_threads.argtypes = [I]
        lib.oracle_set_num_threads.restype = None
        lib.oracle_cost_win.argtypes = [P, P, I, I, I, I, P, P]
        lib.oracle_path_win.argtypes = [P, P, I, I, I, I, I, I, I, P]
        lib.oracle_sgm_win.argtypes = [P, P, I, I, I, I, I, I, I, I, P, P, P]
        lib.oracle_downsample4.argtypes = [P, I, I, I, P]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed (%d)" % (what, rc))


def _dlo(d_lo, H):
    if d_lo is None:
        return None
    d = np.ascontiguousarray(d_lo, dtype=np.int32)
    if d.shape != (H,):
        raise ValueError("d_lo must have one entry per row")
    return d


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loop over path directions (timing only)."""
    _load().oracle_set_num_threads(int(n))


def census(img: np.ndarray, n: int) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.empty((H, W), np.uint64)
    _check(_load().oracle_census(_p(img), W, H, W, n, _p(out)), "census")
    return out


def cost(cl: np.ndarray, cr: np.ndarray, n: int, w: int, d_lo=None) -> np.ndarray:
    cl = np.ascontiguousarray(cl, dtype=np.uint64)
    cr = np.ascontiguousarray(cr, dtype=np.uint64)
    H, W = cl.shape
    d = _dlo(d_lo, H)
    out = np.empty((H, W, w), np.uint8)
    _check(_load().oracle_cost(_p(cl), _p(cr), W, H, n, w, _p(d), _p(out)), "cost")
    return out


def path(c: np.ndarray, r: int, p1: int, p2: int) -> np.ndarray:
    """Normalised aggregated cost L_r (uint16 [H, W, w]) for path index r."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    H, W, w = c.shape
    du, dv = PATHS[r]
    out = np.empty((H, W, w), np.uint16)
    _check(_load().oracle_path(_p(c), W, H, w, du, dv, p1, p2, _p(out)), "path")
    return out


def path_dir(c: np.ndarray, du: int, dv: int, p1: int, p2: int) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.uint8)
    H, W, w = c.shape
    out = np.empty((H, W, w), np.uint16)
    _check(_load().oracle_path(_p(c), W, H, w, du, dv, p1, p2, _p(out)), "path")
    return out


def path_raw(c: np.ndarray, r: int, p1: int, p2: int) -> np.ndarray:
    """Literal eq. (8) without the -min term (int64 [H, W, w])."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    H, W, w = c.shape
    du, dv = PATHS[r]
    out = np.empty((H, W, w), np.int64)
    _check(_load().oracle_path_raw(_p(c), W, H, w, du, dv, p1, p2, _p(out)), "path_raw")
    return out


def sum_paths(c: np.ndarray, npaths: int, p1: int, p2: int) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.uint8)
    H, W, w = c.shape
    out = np.empty((H, W, w), np.uint32)
    _check(_load().oracle_sum(_p(c), W, H, w, npaths, p1, p2, _p(out)), "sum")
    return out


def wta(S: np.ndarray, d_lo=None):
    S = np.ascontiguousarray(S, dtype=np.uint32)
    H, W, w = S.shape
    d = _dlo(d_lo, H)
    dint = np.empty((H, W), np.uint16)
    dsub = np.empty((H, W), np.float32)
    _check(_load().oracle_wta(_p(S), W, H, w, _p(d), _p(dint), _p(dsub)), "wta")
    return dint, dsub


def sgm(left, right, n, w, npaths, p1, p2, d_lo=None):
    """Whole path: returns (Dint uint16 [H,W], Dsub float32 [H,W])."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    H, W = left.shape
    d = _dlo(d_lo, H)
    dint = np.empty((H, W), np.uint16)
    dsub = np.empty((H, W), np.float32)
    _check(_load().oracle_sgm(_p(left), _p(right), W, H, W, n, w, npaths, p1, p2,
                              _p(d), _p(dint), _p(dsub)), "sgm")
    return dint, dsub


def window_from_road(a0, a1, phi, W, H, w, mode=0, delta=0.0) -> np.ndarray:
    """Per-row window start d_lo (int32 [H]); mode 0 centred, 1 eq. (6)."""
    out = np.empty((H,), np.int32)
    _check(_load().oracle_window_from_road(float(a0), float(a1), float(phi), W, H, w,
                                           int(mode), float(delta), _p(out)), "window")
    return out


# ---------------------------------------------------------------------------
# per-pixel windows in absolute disparity


def _lo_map(lo, H, W):
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    if lo.shape != (H, W):
        raise ValueError("lo must be int32 [H, W]")
    return lo


def cost_win(cl, cr, n, w, lo):
    cl = np.ascontiguousarray(cl, dtype=np.uint64)
    cr = np.ascontiguousarray(cr, dtype=np.uint64)
    H, W = cl.shape
    lo = _lo_map(lo, H, W)
    out = np.empty((H, W, w), np.uint8)
    _check(_load().oracle_cost_win(_p(cl), _p(cr), W, H, n, w, _p(lo), _p(out)), "cost_win")
    return out


def path_win(c, lo, r, p1, p2):
    c = np.ascontiguousarray(c, dtype=np.uint8)
    H, W, w = c.shape
    lo = _lo_map(lo, H, W)
    du, dv = PATHS[r]
    out = np.empty((H, W, w), np.uint16)
    _check(_load().oracle_path_win(_p(c), _p(lo), W, H, w, du, dv, p1, p2, _p(out)), "path_win")
    return out


def sgm_win(left, right, n, w, npaths, p1, p2, lo):
    """Per-pixel-window SGM: (Dint uint16, Dsub float32) with D = lo + k*."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    H, W = left.shape
    lo = _lo_map(lo, H, W)
    dint = np.empty((H, W), np.uint16)
    dsub = np.empty((H, W), np.float32)
    _check(_load().oracle_sgm_win(_p(left), _p(right), W, H, W, n, w, npaths, p1, p2, _p(lo),
                                  _p(dint), _p(dsub)), "sgm_win")
    return dint, dsub


def downsample4(img):
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.empty((H // 4, W // 4), np.uint8)
    _check(_load().oracle_downsample4(_p(img), W, H, W, _p(out)), "downsample4")
    return out
