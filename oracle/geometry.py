"""Deformed geometry and variable coefficient (oracle; test infrastructure).

The paper's curved case applies the general cell-wise Laplacian (evaluate
gradients, apply the physics, integrate) with a per-quadrature-point Q_k
mapping (Sec. 6).  This workload replaces the curved ball by the unit cube
under a smooth deformation, with a variable coefficient:

* mapping: x = xh + amp * prod_b sin(2 pi xh_b) * (1, 1, 1), applied at the
  Gauss-Lobatto nodes of every cell and interpolated by Q_k
  (isoparametric); the boundary of the cube stays fixed;
* coefficient: kappa(x) = exp(s * sum_j a_j cos(pi m_j . x + phi_j)) with s
  chosen so that max |exponent| = 1 over the Gauss points of the finest mesh;
* element matrix A_K,ij = sum_q w_q kappa(x_q) det(J_q)
  (J_q^{-T} grad phi_i) . (J_q^{-T} grad phi_j) with a (k+1)^3 Gauss rule;
* load b_K,i = sum_q w_q det(J_q) f(x_q) phi_i(xi_q) with f = 3 pi^2
  prod sin(pi x_a) at the physical points (or a given f), (k+2)^3 Gauss rule.

Everything is evaluated by explicit per-point loops over the Q_k node
values (no sum factorization), in float64.
"""
import numpy as np

from .basis import gauss_legendre, gll_nodes, lagrange_derivatives, lagrange_values


def deform(xh, amp):
    """x = xh + amp * prod_b sin(2 pi xh_b) in every coordinate; xh shape (..., 3)."""
    s = np.prod(np.sin(2 * np.pi * xh), axis=-1)
    return xh + amp * s[..., None]


def cell_node_coords(mesh, amp, cells=None):
    """(n_cells, K^3, 3) physical coordinates of the cells' Q_k geometry nodes
    (all cells, or the listed cell indices)."""
    xi = gll_nodes(mesh.k)
    cc = mesh.cell_coords()
    if cells is not None:
        cc = cc[np.asarray(cells)]
    lc = mesh.local_coords()
    ref = (cc[:, None, :] + xi[lc][None, :, :]) / mesh.n
    return deform(ref, amp)


def tensor_basis(k, pts):
    """Values and reference gradients of the K^3 tensor basis at the tensor grid of pts.

    Returns V (nq^3, K^3) and Gr (nq^3, K^3, 3); point index qx fastest, local
    index ix fastest.
    """
    xi = gll_nodes(k)
    v = lagrange_values(xi, pts)          # (nq, K)
    d = lagrange_derivatives(xi, pts)
    nq, K = len(pts), k + 1
    # point (qx, qy, qz) -> qx + nq*(qy + nq*qz); local (ix, iy, iz) -> ix + K*(iy + K*iz)
    V = np.einsum("xi,yj,zl->zyxlji", v, v, v).reshape(nq ** 3, K ** 3)
    Gx = np.einsum("xi,yj,zl->zyxlji", d, v, v).reshape(nq ** 3, K ** 3)
    Gy = np.einsum("xi,yj,zl->zyxlji", v, d, v).reshape(nq ** 3, K ** 3)
    Gz = np.einsum("xi,yj,zl->zyxlji", v, v, d).reshape(nq ** 3, K ** 3)
    return V, np.stack([Gx, Gy, Gz], axis=-1)


def tensor_weights(w):
    return np.einsum("x,y,z->zyx", w, w, w).ravel()


def coefficient_raw(x, modes, amps, phases):
    """sum_j a_j cos(pi m_j . x + phi_j) at points x (..., 3)."""
    arg = np.pi * np.tensordot(x, modes.T.astype(np.float64), axes=1) + phases
    return np.cos(arg) @ amps


def coefficient_scale(mesh, amp, coef, chunk=2048):
    """s = 1 / max |sum_j a_j cos(pi m_j . x_q + phi_j)| over the (k+1)^3 Gauss
    points x_q of every cell of `mesh`, evaluated chunk by chunk of cells."""
    from concurrent.futures import ThreadPoolExecutor
    modes, amps, phases = (np.asarray(c) for c in coef)
    k = mesh.k
    xq, _ = gauss_legendre(k + 1)
    V, _ = tensor_basis(k, xq)

    def chunk_max(c0):
        X = cell_node_coords(mesh, amp, cells=np.arange(c0, min(mesh.n_cells, c0 + chunk)))
        xphys = np.einsum("qj,ejd->eqd", V, X)
        return float(np.max(np.abs(coefficient_raw(xphys, modes, amps, phases))))

    # chunks are independent; the maximum does not depend on their order
    with ThreadPoolExecutor(max_workers=8) as ex:
        gmax = max(ex.map(chunk_max, range(0, mesh.n_cells, chunk)))
    return 1.0 / gmax


class DeformedGeometry:
    """Quadrature data of the deformed, variable-coefficient problem on one structured mesh
    (all cells, or the listed cell indices; the coefficient scale s is then taken from
    `scale`, which a caller computes over the whole mesh with coefficient_scale)."""

    def __init__(self, mesh, amp, coef, scale=None, cells=None):
        self.mesh, self.amp = mesh, amp
        self.cells = None if cells is None else np.asarray(cells)
        if self.cells is not None and scale is None and coef is not None and len(coef[1]):
            raise ValueError("a cell subset needs the whole-mesh coefficient scale")
        k = mesh.k
        self.xq, self.wq = gauss_legendre(k + 1)
        self.V, self.Gr = tensor_basis(k, self.xq)
        self.W = tensor_weights(self.wq)
        X = cell_node_coords(mesh, amp, cells=self.cells)           # (E, K^3, 3)
        self.X = X
        self.xphys = np.einsum("qj,ejd->eqd", self.V, X)           # (E, Q, 3)
        # J[e, q, d, a] = d x_d / d xi_a
        self.J = np.einsum("qja,ejd->eqda", self.Gr, X)
        self.detJ = np.linalg.det(self.J)
        modes, amps, phases = coef if coef is not None else (np.zeros((0, 3)), np.zeros(0), np.zeros(0))
        if len(amps):
            graw = coefficient_raw(self.xphys, np.asarray(modes), np.asarray(amps), np.asarray(phases))
            self.scale = 1.0 / np.max(np.abs(graw)) if scale is None else scale
            self.kappa = np.exp(self.scale * graw)
        else:
            self.scale = 1.0
            self.kappa = np.ones(self.detJ.shape)
        Jinv = np.linalg.inv(self.J)                                # (E, Q, a, d)
        # metric G = kappa w det(J) J^{-1} J^{-T}  (reference-gradient space)
        self.G = (self.kappa * self.W[None, :] * self.detJ)[..., None, None] * np.einsum(
            "eqad,eqbd->eqab", Jinv, Jinv)

    def element_matrices(self):
        """Dense A_K for every cell: (E, K^3, K^3)."""
        return np.einsum("qia,eqab,qjb->eij", self.Gr, self.G, self.Gr)

    def apply(self, x_cell):
        """y_K = A_K x_K via the quadrature definition (gradients, metric, integrate)."""
        x = np.asarray(x_cell).reshape(self.G.shape[0], -1)
        grad = np.einsum("qja,ej->eqa", self.Gr, x)
        flux = np.einsum("eqab,eqb->eqa", self.G, grad)
        return np.einsum("qia,eqa->ei", self.Gr, flux)

    def diagonal(self):
        return np.einsum("qia,eqab,qib->ei", self.Gr, self.G, self.Gr)

    def load_vector(self, f=None):
        """b_K,i = int_K f phi_i, (k+2)^3 Gauss rule on the reference cell, det J
        at each point.  f: callable on physical points (..., 3); default the
        manufactured source 3 pi^2 prod sin(pi x_a) of u = prod sin(pi x_a)."""
        k = self.mesh.k
        xq, wq = gauss_legendre(k + 2)
        V, Gr = tensor_basis(k, xq)
        W = tensor_weights(wq)
        xp = np.einsum("qj,ejd->eqd", V, self.X)
        J = np.einsum("qja,ejd->eqda", Gr, self.X)
        if f is None:
            fq = 3 * np.pi ** 2 * np.prod(np.sin(np.pi * xp), axis=-1)
        else:
            fq = f(xp)
        return np.einsum("qi,eq->ei", V, fq * np.linalg.det(J) * W[None, :])

    def l2_error(self, u_cell, u_exact):
        """|| u_h - u ||_L2 over the mapped domain, (k+3)^3 Gauss rule: u_h from the
        cell-wise nodal values, u_exact a callable on physical points."""
        k = self.mesh.k
        xq, wq = gauss_legendre(k + 3)
        V, Gr = tensor_basis(k, xq)
        W = tensor_weights(wq)
        xp = np.einsum("qj,ejd->eqd", V, self.X)
        det = np.linalg.det(np.einsum("qja,ejd->eqda", Gr, self.X))
        uh = np.einsum("qj,ej->eq", V, np.asarray(u_cell).reshape(self.X.shape[0], -1))
        return np.sqrt(np.sum(W[None, :] * det * (uh - u_exact(xp)) ** 2))
