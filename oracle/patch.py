"""Vertex-patch additive Schwarz inverse by dense local solves (oracle; test infrastructure).

The paper admits any smoother of the form P = G P_CG G^T (Sec. 2.1,
eq. precond_consistency) and names overlapping vertex-patch smoothers as
such a substitute (Sec. 3.3, Sec. 4.1).  Reading used here: a patch is the
2^d cells around an interior mesh vertex; its unknowns are the (2k-1)^d
global DoFs strictly inside the patch box (homogeneous Dirichlet on the patch
boundary); the patch operator is A_p = R_p A_CG R_p^T; the patches are
summed additively without damping:

    z = G sum_p R_p^T A_p^{-1} R_p G^T r.

The oracle forms every A_p densely and factors it by Cholesky.
"""
import numpy as np
import scipy.linalg as sla


def interior_vertices(mesh):
    """(n_patches, dim) vertex coordinates, x fastest, each in [1, n-1]."""
    r = range(1, mesh.n)
    if mesh.dim == 2:
        return np.array([(vx, vy) for vy in r for vx in r], dtype=np.int64).reshape(-1, 2)
    return np.array([(vx, vy, vz) for vz in r for vy in r for vx in r],
                    dtype=np.int64).reshape(-1, 3)


def patch_dof_indices(mesh):
    """(n_patches, m^d) global DoF indices of each patch interior, x fastest."""
    k, m = mesh.k, 2 * mesh.k - 1
    verts = interior_vertices(mesh)
    off = np.arange(1, m + 1)
    if mesh.dim == 2:
        ox, oy = np.meshgrid(off, off, indexing="xy")
        ox, oy = ox.ravel(), oy.ravel()
        gx = k * (verts[:, 0:1] - 1) + ox[None, :]
        gy = k * (verts[:, 1:2] - 1) + oy[None, :]
        return gx + mesh.N * gy
    oz, oy, ox = np.meshgrid(off, off, off, indexing="ij")
    ox, oy, oz = ox.ravel(), oy.ravel(), oz.ravel()
    gx = k * (verts[:, 0:1] - 1) + ox[None, :]
    gy = k * (verts[:, 1:2] - 1) + oy[None, :]
    gz = k * (verts[:, 2:3] - 1) + oz[None, :]
    return gx + mesh.N * (gy + mesh.N * gz)


def patch_matrices(A_csr, mesh):
    """Dense A_p = R_p A_CG R_p^T for every patch: (n_patches, m^d, m^d)."""
    idx = patch_dof_indices(mesh)
    out = np.empty((idx.shape[0], idx.shape[1], idx.shape[1]))
    for p in range(idx.shape[0]):
        out[p] = A_csr[idx[p]][:, idx[p]].toarray()
    return out


def patch_inverse_global(A_csr, mesh, r_global, shared=False):
    """z_CG = sum_p R_p^T A_p^{-1} R_p r_global with dense Cholesky solves.

    ``shared=True`` forms A_p once from the first patch and reuses it (valid
    when every patch matrix is the same, e.g. a uniform Cartesian mesh);
    the caller is responsible for that being true.
    """
    idx = patch_dof_indices(mesh)
    r_global = np.asarray(r_global, dtype=np.float64)
    z = np.zeros_like(r_global)
    if idx.shape[0] == 0:
        return z
    if shared:
        Ap = A_csr[idx[0]][:, idx[0]].toarray()
        Ainv = sla.cho_solve(sla.cho_factor(Ap), np.eye(Ap.shape[0]))
        W = r_global[idx] @ Ainv.T
        np.add.at(z, idx.ravel(), W.ravel())
        return z
    for p in range(idx.shape[0]):
        Ap = A_csr[idx[p]][:, idx[p]].toarray()
        w = sla.cho_solve(sla.cho_factor(Ap), r_global[idx[p]])
        np.add.at(z, idx[p], w)
    return z


def shared_patch_inverse(mesh):
    """A_p^{-1} of every interior vertex patch of a uniform Cartesian mesh.

    Every interior patch matrix is the same (translation invariance; the patch
    interiors never touch the boundary), so A_p is taken from the one interior
    vertex of a 2^d mesh with the same element matrix and inverted once
    (Cholesky). Rows and columns in the patch's interior order, x fastest.
    """
    from .mesh import StructuredMesh
    from .operators import assemble_csr, element_matrix_cartesian
    small = StructuredMesh(mesh.dim, mesh.k, 2)
    A_small = assemble_csr(small, element_matrix_cartesian(mesh.dim, mesh.k, mesh.h))
    i0 = patch_dof_indices(small)[0]
    Ap = A_small[i0][:, i0].toarray()
    return sla.cho_solve(sla.cho_factor(Ap), np.eye(Ap.shape[0]))


def patch_inverse_cartesian(mesh, r_cell):
    """z = G sum_p R_p^T A_p^{-1} R_p G^T r on a uniform Cartesian mesh of any size,
    the shared A_p^{-1} (shared_patch_inverse) applied to all patches as one
    dense product.
    """
    Ainv = shared_patch_inverse(mesh)
    idx = patch_dof_indices(mesh)
    r_global = mesh.assemble(r_cell)
    z = np.zeros_like(r_global)
    if idx.shape[0]:
        W = r_global[idx] @ Ainv.T
        for j in range(idx.shape[1]):      # for one local offset the patches' DoFs are distinct
            z[idx[:, j]] += W[:, j]
    return mesh.gather(z)


def patch_inverse_cellwise(A_csr, mesh, r_cell, shared=False):
    """z = G sum_p R_p^T A_p^{-1} R_p G^T r (dual cell-wise in, primal cell-wise out)."""
    r_global = mesh.assemble(r_cell)
    return mesh.gather(patch_inverse_global(A_csr, mesh, r_global, shared=shared))


def dofs_per_patch(mesh):
    return (2 * mesh.k - 1) ** mesh.dim


def patch_membership_count(mesh):
    """How many patch interiors contain each global DoF (for tests)."""
    cnt = np.zeros(mesh.n_global, dtype=np.int64)
    for row in patch_dof_indices(mesh):
        cnt[row] += 1
    return cnt

