"""Structured mesh indexing and the gather operator (oracle; test infrastructure).

Cell-wise storage (paper, Sec. 2.1): every cell stores its own copy of each
of its (k+1)^d nodal DoFs.  The gather operator G replicates a global
coefficient into all cell-local copies, G^T sums the copies.

Conventions (the paper leaves ordering open; these are this project's):

* unit square/cube split into n^d cells of side h = 1/n;
* cell index  e = cx + n*cy (+ n^2*cz), x fastest;
* local index i = ix + K*iy (+ K^2*iz), K = k+1, x fastest;
* global node (gx, gy, gz) with g_a = k*c_a + i_a on the (k n + 1)^d grid,
  global index gx + N*gy (+ N^2*gz), N = k n + 1.

G is built here as an explicit scipy sparse matrix.
"""
import numpy as np
import scipy.sparse as sp


class StructuredMesh:
    def __init__(self, dim, k, n):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim, self.k, self.n = dim, k, n
        self.K = k + 1
        self.N = k * n + 1
        self.h = 1.0 / n
        self.n_cells = n ** dim
        self.n_local = self.K ** dim
        self.n_cellwise = self.n_cells * self.n_local
        self.n_global = self.N ** dim

    # -- index maps ---------------------------------------------------
    def cell_coords(self):
        """(n_cells, dim) integer cell coordinates in storage order."""
        e = np.arange(self.n_cells)
        out = [e % self.n, (e // self.n) % self.n]
        if self.dim == 3:
            out.append(e // (self.n * self.n))
        return np.stack(out, axis=1)

    def local_coords(self):
        """(K^d, dim) local node coordinates in storage order."""
        i = np.arange(self.n_local)
        out = [i % self.K, (i // self.K) % self.K]
        if self.dim == 3:
            out.append(i // (self.K * self.K))
        return np.stack(out, axis=1)

    def global_index_map(self):
        """(n_cells, K^d) array: global DoF index of every cell-wise entry."""
        # global coordinate k*c + i per axis, flattened x fastest:
        # sum_a N^a (k c_a + i_a) = (sum_a N^a k c_a) + (sum_a N^a i_a)
        cc = self.cell_coords()
        lc = self.local_coords()
        stride = self.N ** np.arange(self.dim)
        return (self.k * cc @ stride)[:, None] + (lc @ stride)[None, :]

    def global_coords(self):
        """(n_global, dim) integer node coordinates of every global DoF."""
        g = np.arange(self.n_global)
        out = [g % self.N, (g // self.N) % self.N]
        if self.dim == 3:
            out.append(g // (self.N * self.N))
        return np.stack(out, axis=1)

    def boundary_mask_global(self):
        """True for global DoFs on the boundary of the unit square/cube."""
        gc = self.global_coords()
        return np.any((gc == 0) | (gc == self.N - 1), axis=1)

    # -- operators ----------------------------------------------------
    def gather_matrix(self):
        """Sparse G: V_CG -> V_cell (one 1 per row)."""
        cols = self.global_index_map().ravel()
        rows = np.arange(self.n_cellwise)
        data = np.ones(self.n_cellwise)
        return sp.csr_matrix((data, (rows, cols)),
                             shape=(self.n_cellwise, self.n_global))

    def gather(self, x_global):
        """G x: replicate global coefficients into the cell-wise layout."""
        return np.asarray(x_global)[self.global_index_map()]

    def assemble(self, y_cell):
        """G^T y: sum cell-wise copies into global DoFs."""
        y = np.asarray(y_cell, dtype=np.result_type(y_cell, np.float64)).ravel()
        return np.bincount(self.global_index_map().ravel(), weights=y, minlength=self.n_global)

    def valence_global(self):
        """kappa = diag(G^T G): number of cells sharing each global DoF."""
        return np.asarray(self.gather_matrix().sum(axis=0)).ravel()
