"""Assembled geometric multigrid and PCG on uniform hierarchies (oracle; test infrastructure).

Everything acts on assembled vectors over the interior (non-Dirichlet)
global DoFs of each level, i.e. the classical method that the cell-wise
solver is proved equivalent to:

* Hierarchy T_0 < T_1 < ... < T_L by uniform bisection, n_l = n_0 2^l
  (paper, Sec. 3).
* Prolongation P_CG: interpolation of the coarse Q_k function at the fine
  nodes (the natural embedding of nested spaces, Sec. 3); restriction
  R_CG = P_CG^T (Sec. 3.1, lemma on unassembled restriction).
* Classical damped Jacobi u <- u + w D^{-1}(b - A u) (Sec. 4.1, the lemma
  verifying the smoother assumption, with no refinement edge).
* Chebyshev smoother preconditioned by the vertex-patch inverse (degree d,
  interval [lmax/ratio, lmax]; standard Chebyshev semi-iteration).
* V-cycle exactly as Algorithm 1 (pre-smooth, residual, restrict, recurse
  from zero, prolongate and correct, post-smooth; direct solve at l = 0).
* Preconditioned CG (Sec. 4.4); optionally the flexible (Polak-Ribiere)
  beta.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import gll_nodes, lagrange_values
from .mesh import StructuredMesh
from .operators import assemble_csr, element_matrix_cartesian, interior_indices
from .patch import patch_dof_indices


def global_prolongation_1d(k, n_coarse):
    """P1[f, c] = psi_c(x_f): coarse global 1D basis evaluated at fine node positions."""
    n_f = 2 * n_coarse
    nodes = gll_nodes(k)
    Nf, Nc = k * n_f + 1, k * n_coarse + 1
    # physical coordinates of the fine nodes
    xf = np.empty(Nf)
    for e in range(n_f):
        xf[k * e:k * e + k + 1] = (e + nodes) / n_f
    P = np.zeros((Nf, Nc))
    for f in range(Nf):
        s = xf[f] * n_coarse
        e = min(int(np.floor(s)), n_coarse - 1)
        t = s - e
        vals = lagrange_values(nodes, [t])[0]
        P[f, k * e:k * e + k + 1] = vals
    P[np.abs(P) < 1e-15] = 0.0
    return P


class Level:
    def __init__(self, dim, k, n, elem=None):
        self.mesh = StructuredMesh(dim, k, n)
        if elem is None:
            elem = element_matrix_cartesian(dim, k, 1.0 / n)
        self.elem = elem
        self.A_full = assemble_csr(self.mesh, elem)
        self.I = interior_indices(self.mesh)
        self.A = self.A_full[self.I][:, self.I].tocsr()
        self.diag = self.A.diagonal().copy()
        self.n_int = len(self.I)

    # interior <-> full global vectors
    def to_full(self, u_int):
        u = np.zeros(self.mesh.n_global)
        u[self.I] = u_int
        return u

    def to_int(self, u_full):
        return np.asarray(u_full)[self.I]

    def patch_inverse(self, r_int, shared=False):
        """sum_p R_p^T A_p^{-1} R_p r on interior vectors (dense Cholesky per patch)."""
        r = self.to_full(r_int)
        idx = patch_dof_indices(self.mesh)
        z = np.zeros_like(r)
        cache = None
        for p in range(idx.shape[0]):
            if shared and cache is not None:
                Ainv = cache
            else:
                Ap = self.A_full[idx[p]][:, idx[p]].toarray()
                Ainv = sla.cho_solve(sla.cho_factor(Ap), np.eye(Ap.shape[0]))
                if shared:
                    cache = Ainv
            np.add.at(z, idx[p], Ainv @ r[idx[p]])
        return self.to_int(z)


class Hierarchy:
    """Uniform hierarchy with assembled interior operators on every level."""

    def __init__(self, dim, k, n, n_coarse=1, elem_fn=None):
        self.dim, self.k = dim, k
        ns = []
        m = n
        while m >= n_coarse:
            ns.append(m)
            if m == n_coarse or m % 2:
                break
            m //= 2
        ns = ns[::-1]
        if ns[0] != n_coarse:
            raise ValueError("n must be n_coarse * 2^L")
        self.ns = ns
        self.levels = [Level(dim, k, m, None if elem_fn is None else elem_fn(m)) for m in ns]
        self.P = []
        for l in range(1, len(ns)):
            P1 = global_prolongation_1d(k, ns[l - 1])
            P = sp.csr_matrix(P1)
            Pd = P
            for _ in range(dim - 1):
                Pd = sp.kron(P, Pd, format="csr")
            fine, coarse = self.levels[l], self.levels[l - 1]
            self.P.append(Pd[fine.I][:, coarse.I].tocsr())
        c = self.levels[0]
        self.coarse_inv = np.linalg.inv(c.A.toarray()) if c.n_int > 0 else np.zeros((0, 0))

    @property
    def L(self):
        return len(self.levels) - 1


def jacobi_sweep(level, b, u, omega):
    return u + omega * (b - level.A @ u) / level.diag


def chebyshev_sweep(level, b, u, lmax, degree, ratio=20.0, precond=None, u_is_zero=False):
    """Chebyshev semi-iteration for A u = b preconditioned by ``precond`` on [lmax/ratio, lmax]."""
    if precond is None:
        precond = lambda r: level.patch_inverse(r, shared=True)
    beta_ = lmax
    alpha_ = lmax / ratio
    theta = 0.5 * (beta_ + alpha_)
    delta = 0.5 * (beta_ - alpha_)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b.copy() if u_is_zero else b - level.A @ u
    d = precond(r) / theta
    u = u + d
    for _ in range(1, degree):
        r = r - level.A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * precond(r)
        rho = rho_new
        u = u + d
    return u


def vcycle(h, b, smoother, l=None):
    """Algorithm 1 with a zero initial guess; returns the level-l correction."""
    if l is None:
        l = h.L
    if l == 0:
        return h.coarse_inv @ b
    lev = h.levels[l]
    u = np.zeros_like(b)
    u = smoother(lev, l, b, u, True)
    r = b - lev.A @ u
    bc = h.P[l - 1].T @ r
    ec = vcycle(h, bc, smoother, l - 1)
    u = u + h.P[l - 1] @ ec
    u = smoother(lev, l, b, u, False)
    return u


def make_jacobi_smoother(omega, nu_pre=2, nu_post=2):
    def smooth(lev, l, b, u, pre):
        for _ in range(nu_pre if pre else nu_post):
            u = jacobi_sweep(lev, b, u, omega)
        return u
    return smooth


def make_chebyshev_smoother(lmax_per_level, degree=3, ratio=20.0, nu_pre=1, nu_post=1):
    def smooth(lev, l, b, u, pre):
        for s in range(nu_pre if pre else nu_post):
            u = chebyshev_sweep(lev, b, u, lmax_per_level[l], degree, ratio,
                                u_is_zero=(pre and s == 0))
        return u
    return smooth


def pcg(A, b, M, tol=1e-10, maxit=500, x0=None, flexible=False):
    """Preconditioned CG; stops when ||b - A x||_2 <= tol ||b||_2.  Returns (x, iters, history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    if hist[-1] <= tol:
        return x, 0, hist
    z = M(r)
    p = z.copy()
    rho = r @ z
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol:
            return x, it, hist
        z_new = M(r)
        rho_new = r @ z_new
        beta = (rho_new - r @ z) / rho if flexible else rho_new / rho
        z = z_new
        rho = rho_new
        p = z + beta * p
    return x, maxit, hist
