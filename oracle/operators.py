"""Element matrices, assembly, cell-wise apply and DSS (oracle; test infrastructure).

* Cartesian element matrix (paper, Sec. 6, the cube): the operator is the
  symmetric Kronecker sum (D x B x B + B x D x B + B x B x D) scaled by the
  per-cell scalar det(J) J^{-2}, which is h^{d-2} for a cell of side h.
* General element matrix (paper, Sec. 6, the curved case): integrate
  grad(phi_i) . grad(phi_j) with quadrature (see ``geometry``).
* A_CG = G^T A G (paper, Sec. 2.1, eq. constrained_system), in CSR.
* DSS S = G G^T (eq. dss_operator); averaging DSS S_bar = G (G^T G)^{-1} G^T
  (eq. averaging_dss).
"""
import numpy as np
import scipy.sparse as sp

from .basis import mass_1d, stiffness_1d


def element_matrix_cartesian(dim, k, h):
    """h^{d-2} * sum over directions of D in that direction and B elsewhere.

    Local index is x fastest, so with numpy.kron (last factor fastest) the
    x factor is written last.
    """
    B, D = mass_1d(k), stiffness_1d(k)
    if dim == 2:
        A = np.kron(B, D) + np.kron(D, B)
    else:
        A = (np.kron(B, np.kron(B, D)) + np.kron(B, np.kron(D, B))
             + np.kron(D, np.kron(B, B)))
    return h ** (dim - 2) * A


def cell_matrices(mesh, elem):
    """Broadcast a shared element matrix to (n_cells, nl, nl) or check shape."""
    elem = np.asarray(elem, dtype=np.float64)
    if elem.ndim == 2:
        return np.broadcast_to(elem, (mesh.n_cells,) + elem.shape)
    assert elem.shape == (mesh.n_cells, mesh.n_local, mesh.n_local)
    return elem


def apply_cellwise(mesh, elem, x_cell):
    """y_K = A_K x_K for every cell (dense per-cell products)."""
    x = np.asarray(x_cell, dtype=np.float64).reshape(mesh.n_cells, mesh.n_local)
    elem = np.asarray(elem, dtype=np.float64)
    if elem.ndim == 2:
        return x @ elem.T
    return np.einsum("eij,ej->ei", elem, x)


def assemble_csr(mesh, elem):
    """A_CG = G^T blockdiag(A_K) G as a CSR matrix over all global DoFs."""
    idx = mesh.global_index_map()
    nl = mesh.n_local
    rows = np.repeat(idx, nl, axis=1).ravel()
    cols = np.tile(idx, (1, nl)).ravel()
    data = np.asarray(cell_matrices(mesh, elem)).reshape(mesh.n_cells, nl * nl).ravel()
    A = sp.coo_matrix((data, (rows, cols)), shape=(mesh.n_global, mesh.n_global))
    return A.tocsr()


def interior_indices(mesh):
    """Global DoFs not on the Dirichlet boundary."""
    return np.flatnonzero(~mesh.boundary_mask_global())


def dirichlet_block(A, mesh):
    """A_II: the assembled operator restricted to interior DoFs."""
    I = interior_indices(mesh)
    return A[I][:, I].tocsr()


def dss_sum(mesh, v_cell):
    """S v = G G^T v."""
    return mesh.gather(mesh.assemble(v_cell))


def dss_average(mesh, v_cell):
    """S_bar v = G diag(kappa)^{-1} G^T v."""
    return mesh.gather(mesh.assemble(v_cell) / mesh.valence_global())


def boundary_mask_cellwise(mesh):
    """True for every cell-wise copy of a boundary DoF."""
    return mesh.gather(mesh.boundary_mask_global().astype(np.float64)) > 0.5


def apply_dirichlet(mesh, elem, x_cell):
    """Cell-wise apply of the Dirichlet operator: mask input and output boundary copies.

    G^T of the result equals A_II acting on the interior part of the input,
    extended by zero on the boundary.
    """
    m = boundary_mask_cellwise(mesh).reshape(mesh.n_cells, mesh.n_local)
    x = np.where(m, 0.0, np.asarray(x_cell, dtype=np.float64).reshape(m.shape))
    y = apply_cellwise(mesh, elem, x)
    return np.where(m, 0.0, y)
