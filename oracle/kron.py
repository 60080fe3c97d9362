"""Kronecker form of the Cartesian operator and its exact solver (oracle; test infrastructure).

On the uniform Cartesian mesh the assembled Dirichlet operator is a
Kronecker sum of 1D global matrices (paper, Sec. 6, the cube operator):

    A_II = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1      (3D)

with K1 = sum_e D/h and M1 = sum_e h B assembled over the n intervals and
restricted to interior nodes.  The generalized eigenproblem K1 S = M1 S L,
S^T M1 S = I diagonalizes it, which gives the exact discrete solution of
A_II u = b at sizes where CSR assembly does not fit in memory.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import mass_1d, stiffness_1d


def global_1d(k, n, dirichlet=True):
    """(K1, M1) assembled over n intervals of [0, 1], dense float64."""
    h = 1.0 / n
    B, D = mass_1d(k), stiffness_1d(k)
    N = k * n + 1
    K1 = np.zeros((N, N))
    M1 = np.zeros((N, N))
    for e in range(n):
        s = slice(k * e, k * e + k + 1)
        K1[s, s] += D / h
        M1[s, s] += h * B
    if dirichlet:
        K1, M1 = K1[1:-1, 1:-1], M1[1:-1, 1:-1]
    return K1, M1


class KroneckerOperator:
    """Assembled Dirichlet operator on the uniform Cartesian mesh, in factored form."""

    def __init__(self, dim, k, n):
        self.dim, self.k, self.n = dim, k, n
        self.K1, self.M1 = global_1d(k, n, dirichlet=True)
        self.Ks = sp.csr_matrix(self.K1)
        self.Ms = sp.csr_matrix(self.M1)
        self.m = self.K1.shape[0]
        lam, S = sla.eigh(self.K1, self.M1)
        self.lam, self.S = lam, S

    def _axis_apply(self, u, Mat, axis):
        u = np.moveaxis(u, axis, -1)
        sh = u.shape
        out = (Mat @ u.reshape(-1, sh[-1]).T).T.reshape(sh)
        return np.moveaxis(out, -1, axis)

    def apply(self, u_int):
        """A_II u for u over interior nodes (x fastest)."""
        m, d = self.m, self.dim
        u = np.asarray(u_int, dtype=np.float64).reshape((m,) * d)
        out = np.zeros_like(u)
        # axis -1 is x, axis -2 is y, axis 0 is z in 3D
        for a in range(d):
            t = u
            for b in range(d):
                t = self._axis_apply(t, self.Ks if a == b else self.Ms, b)
            out += t
        return out.ravel()

    def solve(self, b_int):
        """Exact A_II^{-1} b by fast diagonalization with the global 1D eigenpairs."""
        m, d = self.m, self.dim
        t = np.asarray(b_int, dtype=np.float64).reshape((m,) * d)
        for a in range(d):
            t = self._axis_apply(t, self.S.T, a)
        lam = self.lam
        if d == 2:
            den = lam[:, None] + lam[None, :]
        else:
            den = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
        t = t / den
        for a in range(d):
            t = self._axis_apply(t, self.S, a)
        return t.ravel()

    def min_eigenvalue(self):
        """Smallest generalized eigenvalue of (A_II, M_II): d * lambda_min(K1, M1)."""
        return self.dim * self.lam[0]
