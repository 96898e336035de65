"""ctypes wrapper of the oracle's naive matrix-free apply and diagonal (naive.c).

Test infrastructure only (see the package docstring).
"""
import ctypes
import os

import numpy as np

from . import build as _build
from . import gll

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        args = [ctypes.c_int] * 4 + [dp, dp, dp, ip, dp, dp, ctypes.c_double, dp, ctypes.c_double, dp]
        L.oracle_apply.argtypes = args + [dp]
        L.oracle_apply.restype = ctypes.c_int
        L.oracle_diag.argtypes = args
        L.oracle_diag.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Operator:
    """y = (lambda M + K_nu) x on a mesh spec (see synth.mesh_spec)."""

    def __init__(self, spec, lam, nu=1.0):
        self.spec = spec
        self.lam = float(lam)
        self.P = spec["P"]
        self.nx, self.ny, self.nz = spec["nx"], spec["ny"], spec["nz"]
        self.N = self.nx * self.ny * self.nz * (self.P + 1) ** 3
        self.xv = np.ascontiguousarray(spec["xv"], dtype=np.float64)
        self.yv = np.ascontiguousarray(spec["yv"], dtype=np.float64)
        self.zv = np.ascontiguousarray(spec["zv"], dtype=np.float64)
        self.bc = np.ascontiguousarray(spec["bc"], dtype=np.int32)
        self.D = np.ascontiguousarray(gll.diff_matrix(self.P))
        self.w = np.ascontiguousarray(gll.weights(self.P))
        if np.isscalar(nu):
            self.nu_field, self.nu_const = None, float(nu)
        else:
            self.nu_field = np.ascontiguousarray(nu, dtype=np.float64)
            assert self.nu_field.shape == (self.N,)
            self.nu_const = 0.0

    def _common(self):
        return (self.nx, self.ny, self.nz, self.P, _p(self.xv), _p(self.yv), _p(self.zv),
                self.bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(self.D), _p(self.w),
                self.lam, None if self.nu_field is None else _p(self.nu_field), self.nu_const)

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.N,)
        y = np.empty_like(x)
        rc = lib().oracle_apply(*self._common(), _p(x), _p(y))
        if rc != 0:
            raise ValueError("oracle_apply failed")
        return y

    def diag(self):
        d = np.empty(self.N)
        rc = lib().oracle_diag(*self._common(), _p(d))
        if rc != 0:
            raise ValueError("oracle_diag failed")
        return d


def num_threads():
    return lib().oracle_num_threads()
