"""The plain C FP64 reference (oracle/csrc/fe_oracle.c) of the Cartesian
cell-wise Dirichlet apply and the vertex-patch inverse, for the CPU baseline
at full benchmark sizes.

Test infrastructure like the rest of the oracle: only tests and the
benchmark's CPU baseline load it. It computes the same definitions as
`operators.apply_dirichlet` and `patch.patch_inverse_cartesian` (pinned
against them in tests/test_oracle_c.py), one OpenMP thread per independent
output; the element matrix and the shared patch inverse come from the numpy
oracle.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "fe_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle_c.so")


def build():
    """Compile the C oracle (gcc, OpenMP)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_apply_dirichlet.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_apply_dirichlet.restype = None
        L.oracle_patch_inverse.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        L.oracle_patch_inverse.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads():
    return int(lib().oracle_max_threads())


class CartesianOracle:
    """Apply and patch inverse of the 3D uniform Cartesian Q_k mesh with n^3 cells."""

    def __init__(self, mesh):
        from .operators import element_matrix_cartesian
        from .patch import shared_patch_inverse
        if mesh.dim != 3 or not 1 <= mesh.k <= 8:
            raise ValueError("the C oracle covers 3D meshes with 1 <= k <= 8")
        self.mesh = mesh
        self.k, self.n = mesh.k, mesh.n
        self.A = np.ascontiguousarray(element_matrix_cartesian(3, mesh.k, mesh.h), dtype=np.float64)
        self.Ainv = np.ascontiguousarray(shared_patch_inverse(mesh), dtype=np.float64)
        N = mesh.k * mesh.n + 1
        self.g = np.empty(N ** 3)
        self.zg = np.empty(N ** 3)
        self.W = np.empty(max(mesh.n - 1, 0) ** 3 * (2 * mesh.k - 1) ** 3)

    def apply_dirichlet(self, x_cell, out=None):
        x = np.ascontiguousarray(x_cell, dtype=np.float64).reshape(-1)
        y = np.empty_like(x) if out is None else out
        lib().oracle_apply_dirichlet(self.k, self.n, _ptr(self.A), _ptr(x), _ptr(y))
        return y

    def patch_inverse(self, r_cell, out=None):
        r = np.ascontiguousarray(r_cell, dtype=np.float64).reshape(-1)
        z = np.empty_like(r) if out is None else out
        lib().oracle_patch_inverse(self.k, self.n, _ptr(self.Ainv), _ptr(r), _ptr(z), _ptr(self.g), _ptr(self.zg),
                                   _ptr(self.W))
        return z
