"""Separable (Kronecker-sum) patch surrogates on the deformed mesh (oracle; test infrastructure).

Reading used here (the paper has no deformed patch smoother; its admissible
smoother class is eq. precond_consistency): a patch operator is replaced by

    A_sep = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz,

with per-direction two-interval 1D matrices K_d = alpha_{d,0} D on the
first interval + alpha_{d,1} D on the second, M_d likewise with beta_{d,c}
and B (reference matrices on [0, 1], interior nodes only).  The weights are

* averaged geometry: least squares in log space so that
  alpha_{d,s_d} prod_{e != d} beta_{e,s_e} matches the diagonal entry G_dd of
  the cell-averaged metric of cell s (24 equations, 12 unknowns,
  minimum-norm solution);
* best Kronecker-sum fit: minimize ||A_p - A_sep(theta)||_F over the 12
  weights by alternating linear least squares (see ``best_fit``).

The surrogate inverse is applied densely: z = G sum_p R_p^T A_sep,p^{-1} R_p G^T r.
"""
import numpy as np

from .basis import mass_1d, stiffness_1d
from .patch import interior_vertices, patch_dof_indices


def design_matrix():
    """(24, 12) matrix of the log-space fit; row d*8 + s, s = sx + 2 sy + 4 sz."""
    A = np.zeros((24, 12))
    for d in range(3):
        for s in range(8):
            sl = (s & 1, (s >> 1) & 1, s >> 2)
            r = d * 8 + s
            A[r, 2 * d + sl[d]] = 1.0
            for e in range(3):
                if e != d:
                    A[r, 6 + 2 * e + sl[e]] = 1.0
    return A


def patch_cells(mesh):
    """(n_patches, 8) cell indices of each patch, slot s = sx + 2 sy + 4 sz."""
    v = interior_vertices(mesh)
    out = np.empty((len(v), 8), dtype=np.int64)
    n = mesh.n
    for s in range(8):
        cx = v[:, 0] - 1 + (s & 1)
        cy = v[:, 1] - 1 + ((s >> 1) & 1)
        cz = v[:, 2] - 1 + (s >> 2)
        out[:, s] = cx + n * (cy + n * cz)
    return out


def averaged_weights(geom):
    """(n_patches, 12) weights [alpha_x0, alpha_x1, ..., alpha_z1, beta_x0, ..., beta_z1]."""
    gbar = np.stack([geom.G[:, :, d, d].sum(axis=1) for d in range(3)], axis=1)   # (E, 3)
    cells = patch_cells(geom.mesh)
    lg = np.log(gbar[cells])                  # (P, 8, 3)
    rhs = np.transpose(lg, (0, 2, 1)).reshape(len(cells), 24)
    theta = rhs @ np.linalg.pinv(design_matrix()).T
    return np.exp(theta)


def one_d_factors(k, w):
    """(K_d, M_d) interior two-interval matrices for alpha = w[:2], beta = w[2:]."""
    B, D = mass_1d(k), stiffness_1d(k)
    N = 2 * k + 1
    Kd, Md = np.zeros((N, N)), np.zeros((N, N))
    for e in range(2):
        s = slice(k * e, k * e + k + 1)
        Kd[s, s] += w[e] * D
        Md[s, s] += w[2 + e] * B
    return Kd[1:-1, 1:-1], Md[1:-1, 1:-1]


def sep_matrix(k, weights):
    """Dense A_sep for one patch (local index x fastest)."""
    f = [one_d_factors(k, [weights[2 * d], weights[2 * d + 1], weights[6 + 2 * d], weights[7 + 2 * d]])
         for d in range(3)]
    (Kx, Mx), (Ky, My), (Kz, Mz) = f
    return (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx)))


def sep_patch_inverse_cellwise(mesh, weights, r_cell):
    """z = G sum_p R_p^T A_sep,p^{-1} R_p G^T r with dense solves."""
    idx = patch_dof_indices(mesh)
    rg = mesh.assemble(r_cell)
    z = np.zeros_like(rg)
    for p in range(idx.shape[0]):
        w = np.linalg.solve(sep_matrix(mesh.k, weights[p]), rg[idx[p]])
        np.add.at(z, idx[p], w)
    return mesh.gather(z)
