"""Manufactured right-hand side (oracle; test infrastructure).

Model problem (paper, Sec. 2, eq. poisson): -Laplace u = f with homogeneous
Dirichlet data.  The manufactured solution is u = prod_a sin(pi x_a), so
f = d pi^2 u.  The unassembled load vector is b_K,i = int_K f phi_i, which
the oracle integrates with a (k+2)^d Gauss-Legendre rule on each Cartesian
cell.
"""
import numpy as np

from .basis import gauss_legendre, gll_nodes, lagrange_values


def exact_solution(x):
    """u(x) = prod sin(pi x_a); x has shape (..., d)."""
    return np.prod(np.sin(np.pi * x), axis=-1)


def load_vector_cartesian(mesh):
    """Cell-wise dual vector b_K,i = int_K f phi_i, shape (n_cells, K^d)."""
    k, d, h = mesh.k, mesh.dim, mesh.h
    xq, wq = gauss_legendre(k + 2)
    V = lagrange_values(gll_nodes(k), xq)            # (nq, K)
    cc = mesh.cell_coords()
    out = np.empty((mesh.n_cells, mesh.n_local))
    for e in range(mesh.n_cells):
        # separable integrand: f = d pi^2 prod sin(pi x_a)
        fac = []
        for a in range(d):
            xa = (cc[e, a] + xq) * h
            fac.append(V.T @ (wq * h * np.sin(np.pi * xa)))   # (K,)
        if d == 2:
            blk = np.outer(fac[1], fac[0])
        else:
            blk = np.einsum("i,j,l->ijl", fac[2], fac[1], fac[0])
        out[e] = d * np.pi ** 2 * blk.ravel()
    return out


def l2_error_cartesian(mesh, u_cell):
    """|| u_h - u ||_{L2} with a (k+3)^d Gauss rule per cell."""
    k, d, h = mesh.k, mesh.dim, mesh.h
    xq, wq = gauss_legendre(k + 3)
    V = lagrange_values(gll_nodes(k), xq)
    cc = mesh.cell_coords()
    u = np.asarray(u_cell).reshape(mesh.n_cells, *(mesh.K,) * d)
    err2 = 0.0
    for e in range(mesh.n_cells):
        if d == 2:
            uh = np.einsum("qj,pi,ji->qp", V, V, u[e])       # (qy, qx)
            X, Y = np.meshgrid((cc[e, 0] + xq) * h, (cc[e, 1] + xq) * h, indexing="xy")
            ue = np.sin(np.pi * X) * np.sin(np.pi * Y)
            w = np.outer(wq, wq) * h * h
        else:
            uh = np.einsum("rl,qj,pi,lji->rqp", V, V, V, u[e])
            Z, Y, X = np.meshgrid((cc[e, 2] + xq) * h, (cc[e, 1] + xq) * h,
                                  (cc[e, 0] + xq) * h, indexing="ij")
            ue = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
            w = np.einsum("a,b,c->abc", wq, wq, wq) * h ** 3
        err2 += np.sum(w * (uh - ue) ** 2)
    return np.sqrt(err2)
