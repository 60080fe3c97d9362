"""Locally refined hierarchy and the classical local multigrid (oracle; test infrastructure).

Paper, Sec. 3.2 (adaptive multigrid and edge constraints).  Every cell of
the unit cube may be split isotropically into 2^3 children, recursively; the
leaves form the active mesh T_act.  The level mesh T_l is the set of ALL
level-l cells, active or refined further; it covers the subdomain Omega_l.
This module builds, from plain definitions and with assembled matrices:

* the refinement tree (a fixed rule, shared with the library only as a
  description: refine every cell of the first `global_refinements` levels,
  then, for `adaptive_refinements` more levels, the cells near a feature),
  made 2:1 balanced across faces, edges and vertices;
* per level: the conforming Q_k space on T_l (nodes of all level-l cells),
  the gather G_l, A_l = G_l^T blockdiag(A_K) G_l, the Dirichlet nodes on the
  boundary of the cube, and the partition of the other nodes into the
  refinement edge E_l (nodes on the boundary of Omega_l that are inside the
  cube) and the interior S_l (Sec. 3.2.1);
* the classical prolongation P_CG (coarse Q_k basis evaluated at the fine
  nodes; the natural embedding), restriction P_CG^T;
* the active-mesh space with hanging-node constraints written out as a
  matrix (free nodes -> all node copies of the active cells), the constrained
  system C^T A C (eq. constrained_system) and its exact solution;
* the classical local V-cycle of Algorithm 5 in assembled form: damped
  Jacobi on S_l with E_l frozen (the lemma verifying the smoother
  assumption), residual restriction through P_CG^T (which equals
  R_CG C_HN^T for any constraint operator with C_HN P_CG = P_CG, the lemma on
  the residual transfer), direct coarse solve; the level distribution
  (eq. level_distribution) and the reassembly (eq. level_gather) of
  Algorithm 4, which make it a preconditioner for the active system.

Canonical cell order (the library stores its levels in the same order):
level 0 is the single cell (0, 0, 0); level l lists, for each refined cell
of level l-1 in order, its 8 children c = bx + 2 by + 4 bz at coordinates
2 * parent + (bx, by, bz).  Cell-wise vectors of the active mesh are kept in
"level layout": the level-l blocks concatenated, with zeros on refined cells.
"""
import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import gll_nodes, lagrange_values
from .operators import element_matrix_cartesian

FEATURE_SPHERE, FEATURE_POINT = 0, 1
CHILD_BITS = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)])
NEIGHBOR_OFFSETS = np.array([d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)])


# ------------------------------------------------------------------ tree

def feature_marks(coords, level, feature, center, radius, band):
    """Refinement predicate on the cells of one level: the cell centre lies within
    band * h of the feature (a sphere surface of the given centre and radius, or
    the point `center`).  Squared distances keep the test exact for dyadic data."""
    h = 0.5 ** level
    c = (coords + 0.5) * h
    d2 = np.sum((c - np.asarray(center, dtype=np.float64)) ** 2, axis=1)
    bh = band * h
    if feature == FEATURE_SPHERE:
        lo = max(radius - bh, 0.0)
        return (d2 >= lo * lo) & (d2 <= (radius + bh) * (radius + bh))
    if feature == FEATURE_POINT:
        return d2 <= bh * bh
    raise ValueError("unknown feature")


class RefinementTree:
    """Octree over the unit cube with 2:1 balance (face, edge and vertex neighbours)."""

    def __init__(self, global_refinements, adaptive_refinements, feature=FEATURE_SPHERE,
                 center=(0.5, 0.5, 0.5), radius=0.3125, band=1.0):
        g, a = global_refinements, adaptive_refinements
        L = g + a
        present = [{(0, 0, 0)}]
        refined = []
        for l in range(L):
            cells = np.array(sorted(present[l]), dtype=np.int64).reshape(-1, 3)
            if l < g:
                mark = np.ones(len(cells), dtype=bool)
            else:
                mark = feature_marks(cells, l, feature, center, radius, band)
            refined.append({tuple(c) for c in cells[mark]})
            present.append({tuple(2 * np.array(c) + b) for c in refined[l] for b in CHILD_BITS})
        refined.append(set())
        # balance: a refined level-l cell needs all 26 level-l neighbours to exist
        self.balance_added = 0
        for l in range(L - 1, 0, -1):
            n_l = 2 ** l
            for c in list(refined[l]):
                for d in NEIGHBOR_OFFSETS:
                    nb = tuple(np.array(c) + d)
                    if min(nb) < 0 or max(nb) >= n_l or nb in present[l]:
                        continue
                    par = tuple(np.array(nb) // 2)
                    self.balance_added += par not in refined[l - 1]
                    refined[l - 1].add(par)
                    for b in CHILD_BITS:
                        present[l].add(tuple(2 * np.array(par) + b))
        # drop empty finest levels, then the canonical order
        while len(refined) > 1 and not refined[-2]:
            refined.pop()
            present.pop()
        self.L = len(present) - 1
        self.coords, self.refined = [], []
        order = [np.zeros((1, 3), dtype=np.int64)]
        for l in range(self.L + 1):
            if l > 0:
                prev = self.coords[l - 1]
                par = prev[self.refined[l - 1]]
                order.append((2 * par[:, None, :] + CHILD_BITS[None, :, :]).reshape(-1, 3))
            cc = order[l]
            assert {tuple(c) for c in cc} == present[l], "tree is not closed under the canonical order"
            self.coords.append(cc)
            self.refined.append(np.array([tuple(c) in refined[l] for c in cc], dtype=bool))
        self.index = [{tuple(c): i for i, c in enumerate(cc)} for cc in self.coords]

    def n_cells(self, l):
        return len(self.coords[l])

    def active(self, l):
        return ~self.refined[l]

    def check_balance(self):
        """Every refined cell's 26 level neighbours exist (True if 2:1 balanced)."""
        for l in range(1, self.L + 1):
            n_l = 2 ** l
            for c in self.coords[l][self.refined[l]]:
                for d in NEIGHBOR_OFFSETS:
                    nb = tuple(c + d)
                    if min(nb) >= 0 and max(nb) < n_l and nb not in self.index[l]:
                        return False
        return True


# ------------------------------------------------------------------ level spaces

class LevelSpace:
    """Conforming Q_k space on the level mesh T_l (all level-l cells)."""

    def __init__(self, tree, l, k):
        self.l, self.k, self.K = l, k, k + 1
        K = self.K
        cc = tree.coords[l]
        self.n_cells = len(cc)
        self.h = 0.5 ** l
        self.N = k * 2 ** l + 1                       # node lattice per axis
        loc = np.array([[i % K, (i // K) % K, i // (K * K)] for i in range(K ** 3)])
        lat = k * cc[:, None, :] + loc[None, :, :]    # (cells, K^3, 3) lattice coordinates
        key = (lat[..., 2] * self.N + lat[..., 1]) * self.N + lat[..., 0]
        self.node_keys, inv = np.unique(key.ravel(), return_inverse=True)
        self.copy_node = inv.reshape(self.n_cells, K ** 3)
        self.n_nodes = len(self.node_keys)
        nl = self.node_keys
        self.node_lat = np.stack([nl % self.N, (nl // self.N) % self.N, nl // (self.N * self.N)], axis=1)
        rows = np.arange(self.n_cells * K ** 3)
        self.G = sp.csr_matrix((np.ones(len(rows)), (rows, self.copy_node.ravel())),
                               shape=(len(rows), self.n_nodes))
        Ae = element_matrix_cartesian(3, k, self.h)
        self.A = (self.G.T @ sp.block_diag([Ae] * self.n_cells, format="csr") @ self.G).tocsr()
        self.boundary = np.any((self.node_lat == 0) | (self.node_lat == self.N - 1), axis=1)
        # refinement edge: a node inside the cube whose surrounding lattice cells are
        # not all level-l cells (it lies on the boundary of Omega_l)
        present = tree.index[l]
        n_l = 2 ** l
        edge = np.zeros(self.n_nodes, dtype=bool)
        for j in np.flatnonzero(~self.boundary):
            cand = []
            for a in range(3):
                g = self.node_lat[j, a]
                q, r = divmod(int(g), k)
                cand.append([q - 1, q] if r == 0 else [q])
            for c in itertools.product(*cand):
                if min(c) >= 0 and max(c) < n_l and c not in present:
                    edge[j] = True
                    break
        self.edge = edge
        self.interior = ~self.boundary & ~edge          # S_l
        self.diag = self.A.diagonal().copy()

    def node_positions(self):
        """Physical coordinates of the level nodes."""
        xi = gll_nodes(self.k)
        q = np.minimum(self.node_lat // self.k, 2 ** self.l - 1)
        r = self.node_lat - self.k * q
        return (q + xi[r]) * self.h


def prolongation(tree, coarse, fine):
    """P_CG from level l-1 nodes to level l nodes: the coarse Q_k basis of the
    parent cell evaluated at each fine node (the natural embedding)."""
    k = fine.k
    xi = gll_nodes(k)
    x = fine.node_positions()
    # a level-l cell containing each fine node (the cell of its first copy), its parent
    _, first = np.unique(fine.copy_node.ravel(), return_index=True)
    e = first // (k + 1) ** 3
    par = tree.coords[fine.l][e] // 2
    pe = np.array([tree.index[coarse.l][tuple(c)] for c in par])
    t = x / coarse.h - par                                   # reference coordinates in the parent
    vx, vy, vz = (lagrange_values(xi, t[:, a]) for a in range(3))
    w = np.einsum("ni,nj,nl->nlji", vx, vy, vz).reshape(len(x), -1)   # local index x fastest
    cols = coarse.copy_node[pe]
    w[np.abs(w) < 1e-15] = 0.0
    P = sp.csr_matrix((w.ravel(), (np.repeat(np.arange(len(x)), w.shape[1]), cols.ravel())),
                      shape=(fine.n_nodes, coarse.n_nodes))
    P.eliminate_zeros()
    return P


# ------------------------------------------------------------------ active-mesh system

class ActiveSystem:
    """Continuous Q_k on the active mesh with hanging nodes constrained to the
    coarse side (constraint matrix written out), Dirichlet or free boundary."""

    def __init__(self, tree, k, dirichlet=True):
        self.tree, self.k, self.K = tree, k, k + 1
        K = self.K
        xi = gll_nodes(k)
        loc = np.array([[i % K, (i // K) % K, i // (K * K)] for i in range(K ** 3)])
        cells = [(l, e) for l in range(tree.L + 1) for e in np.flatnonzero(tree.active(l))]
        self.cells = cells
        lo = np.array([tree.coords[l][e] * 0.5 ** l for l, e in cells])
        size = np.array([0.5 ** l for l, _ in cells])
        pos = lo[:, None, :] + xi[loc][None, :, :] * size[:, None, None]      # (cells, K^3, 3)
        keys = np.round(pos * 2 ** 40).astype(np.int64)
        flat = keys.reshape(-1, 3)
        uniq, inv = np.unique(flat, axis=0, return_inverse=True)
        inv = inv.ravel()
        self.copy_node = inv.reshape(len(cells), K ** 3)
        n_all = len(uniq)
        node_pos = np.zeros((n_all, 3))
        node_pos[inv] = pos.reshape(-1, 3)
        self.node_pos = node_pos
        # constraints: a node is hanging when one of the coarsest active cells that
        # contain it in their closure does not have it as a node; its value is then
        # that cell's field there (the coarse side is the master)
        cell_level = np.array([l for l, _ in cells])
        eps = 1e-12
        is_node = sp.csr_matrix((np.ones(self.copy_node.size, dtype=bool),
                                 (np.repeat(np.arange(len(cells)), K ** 3), self.copy_node.ravel())),
                                shape=(len(cells), n_all)).toarray()
        inside = np.ones((len(cells), n_all), dtype=bool)
        for a in range(3):
            inside &= (lo[:, a:a + 1] <= node_pos[None, :, a] + eps)
            inside &= (node_pos[None, :, a] <= lo[:, a:a + 1] + size[:, None] + eps)
        lvl = np.where(inside, cell_level[:, None], 1 << 30)
        coarsest = inside & (lvl == lvl.min(axis=0)[None, :])
        master = coarsest & ~is_node
        hang = np.flatnonzero(master.any(axis=0))
        mcell = np.argmax(master[:, hang], axis=0)
        t = (node_pos[hang] - lo[mcell]) / size[mcell][:, None]
        vx, vy, vz = (lagrange_values(xi, t[:, a]) for a in range(3))
        w = np.einsum("ni,nj,nl->nlji", vx, vy, vz).reshape(len(hang), -1)
        w[np.abs(w) < 1e-14] = 0.0
        # M: all nodes <- all nodes (identity on the others); resolve chains by powers
        keep = np.ones(n_all, dtype=bool)
        keep[hang] = False
        ident = np.flatnonzero(keep)
        rows = np.concatenate([ident, np.repeat(hang, K ** 3)])
        cols = np.concatenate([ident, self.copy_node[mcell].ravel()])
        vals = np.concatenate([np.ones(len(ident)), w.ravel()])
        M = sp.csr_matrix((vals, (rows, cols)), shape=(n_all, n_all))
        M.eliminate_zeros()
        for _ in range(8):
            M2 = (M @ M).tocsr()
            M2.eliminate_zeros()
            if abs(M2 - M).max() < 1e-15:
                break
            M = M2
        else:
            raise AssertionError("constraint chains did not resolve")
        assert M[:, hang].nnz == 0, "a hanging node supports another"
        self.hanging = np.zeros(n_all, dtype=bool)
        self.hanging[hang] = True
        on_bnd = np.any((node_pos < eps) | (node_pos > 1 - eps), axis=1)
        free = ~self.hanging & (~on_bnd if dirichlet else np.ones(n_all, dtype=bool))
        self.free = np.flatnonzero(free)
        # C: all active nodes <- free nodes (columns of M at the free nodes)
        self.C = M[:, self.free].tocsr()
        ncopy = len(cells) * K ** 3
        Gall = sp.csr_matrix((np.ones(ncopy), (np.arange(ncopy), inv)), shape=(ncopy, n_all))
        self.G = (Gall @ self.C).tocsr()                  # active copies <- free DoFs
        blocks = [element_matrix_cartesian(3, k, 0.5 ** l) for l, _ in cells]
        self.A_cells = sp.block_diag(blocks, format="csr")
        self.A = (self.G.T @ self.A_cells @ self.G).tocsr()

    # level layout <-> active copies
    def from_level_layout(self, v, spaces):
        out = np.zeros((len(self.cells), self.K ** 3))
        offs = level_offsets(spaces)
        for i, (l, e) in enumerate(self.cells):
            out[i] = v[offs[l] + e * self.K ** 3: offs[l] + (e + 1) * self.K ** 3]
        return out.ravel()

    def to_level_layout(self, w, spaces):
        offs = level_offsets(spaces)
        v = np.zeros(offs[-1])
        w = np.asarray(w).reshape(len(self.cells), -1)
        for i, (l, e) in enumerate(self.cells):
            v[offs[l] + e * self.K ** 3: offs[l] + (e + 1) * self.K ** 3] = w[i]
        return v

    def solve(self, b_copies):
        """Exact discrete solution of C^T A C u = C^T b, returned at the active copies."""
        u = sla.solve(self.A.toarray(), self.G.T @ b_copies, assume_a="pos")
        return self.G @ u


def level_offsets(spaces):
    offs = [0]
    for s in spaces:
        offs.append(offs[-1] + s.n_cells * s.K ** 3)
    return offs


# ------------------------------------------------------------------ classical local multigrid

class LocalMultigrid:
    """Algorithms 4 and 5 in classical assembled form (Janssen-Kanschat local smoothing)."""

    def __init__(self, tree, k, omega=0.7, nu_pre=1, nu_post=1):
        self.tree, self.k, self.K = tree, k, k + 1
        self.omega, self.nu_pre, self.nu_post = omega, nu_pre, nu_post
        self.spaces = [LevelSpace(tree, l, k) for l in range(tree.L + 1)]
        self.P = [None] + [prolongation(tree, self.spaces[l - 1], self.spaces[l]) for l in range(1, tree.L + 1)]
        c = self.spaces[0]
        self.coarse_int = np.flatnonzero(~c.boundary)
        Ac = c.A[self.coarse_int][:, self.coarse_int].toarray()
        self.coarse_inv = np.linalg.inv(Ac) if len(self.coarse_int) else np.zeros((0, 0))
        self.offsets = level_offsets(self.spaces)

    def smooth(self, l, b, u, sweeps):
        s = self.spaces[l]
        S = s.interior
        for _ in range(sweeps):
            r = b - s.A @ u
            u = u.copy()
            u[S] += self.omega * r[S] / s.diag[S]
        return u

    def vcycle(self, l, b, u):
        """MG_local(A_l, b_l, u_l, l): b[l] and u[l] are the shared level states."""
        s = self.spaces[l]
        if l == 0:
            u[0] = np.zeros(s.n_nodes)
            u[0][self.coarse_int] = self.coarse_inv @ b[0][self.coarse_int]
            return
        u[l] = self.smooth(l, b[l], u[l], self.nu_pre)
        r = b[l] - s.A @ u[l]
        r[s.boundary] = 0.0
        b[l - 1] = b[l - 1] + self.P[l].T @ r
        self.vcycle(l - 1, b, u)
        u[l] = u[l] + self.P[l] @ u[l - 1]
        u[l] = self.smooth(l, b[l], u[l], self.nu_post)

    def precondition(self, r_level_layout):
        """Algorithm 4 from a zero iterate: the unassembled active residual (level
        layout, zeros on refined cells) -> the correction on the active copies
        (level layout, zeros on refined cells)."""
        K3 = self.K ** 3
        b, u = [], []
        for l, s in enumerate(self.spaces):
            rl = np.asarray(r_level_layout[self.offsets[l]:self.offsets[l + 1]]).reshape(s.n_cells, K3).copy()
            rl[self.tree.refined[l]] = 0.0                 # level distribution
            bl = s.G.T @ rl.ravel()
            bl[s.boundary] = 0.0
            b.append(bl)
            u.append(np.zeros(s.n_nodes))
        self.vcycle(self.tree.L, b, u)
        out = np.zeros(self.offsets[-1])
        for l, s in enumerate(self.spaces):
            el = (s.G @ u[l]).reshape(s.n_cells, K3)
            el[self.tree.refined[l]] = 0.0                  # reassembly: active components only
            out[self.offsets[l]:self.offsets[l + 1]] = el.ravel()
        return out

    def edge_mask_copies(self, l):
        """Refinement-edge flag of every cell-wise entry of level l."""
        s = self.spaces[l]
        return s.edge[s.copy_node].ravel()


def load_vector_level_layout(tree, spaces, k):
    """b_K,i = int_K f phi_i on the active cells (f = 3 pi^2 prod sin(pi x_a),
    (k+2)-point Gauss rule per direction), zeros on refined cells; level layout."""
    from .basis import gauss_legendre
    xq, wq = gauss_legendre(k + 2)
    V = lagrange_values(gll_nodes(k), xq)            # (nq, K)
    out = []
    for l, s in enumerate(spaces):
        h = 0.5 ** l
        blk = np.zeros((s.n_cells, (k + 1) ** 3))
        for e in np.flatnonzero(tree.active(l)):
            c = tree.coords[l][e]
            fac = [V.T @ (wq * h * np.sin(np.pi * (c[a] + xq) * h)) for a in range(3)]
            blk[e] = 3 * np.pi ** 2 * np.einsum("i,j,l->lji", fac[0], fac[1], fac[2]).ravel()
        out.append(blk.ravel())
    return np.concatenate(out)
