"""Multi-block mesh and its direct stiffness summation (oracle; test infrastructure).

Paper, Sec. 4.3 (unstructured inter-block interfaces, Algorithm 8): within a
structured macro-block DSS is the axis cascade; across macro-blocks the
shared DoFs are summed by face, line and vertex passes.  The oracle does not
follow those passes: it numbers the global nodes of the whole mesh from their
positions and forms S = G G^T with an explicit sparse G, the definition of
DSS (eq. dss_operator).

The synthetic mesh is a 7-block "ball atlas" in its piecewise-bilinear form
(the curved ball of the paper is not available): a centre cube [-1, 1]^3 and
six caps between the cube's faces and the faces of [-2, 2]^3 (each cap a
frustum over one cube face), so macro-faces join 2 blocks, macro-lines 2 or
3 and macro-vertices 3 or 4.  Each block is an n^3 grid of Q_k cells with its
own orientation: block-local lattice coordinates a_d in [0, kn] give
t_d = a_{perm[d]} (or kn - a_{perm[d]} when flipped), and with m = kn

* centre:       X = (2 t - m) m
* cap (axis e, sign s):  X_e = s (m + t_0) m,
                         X_f = (m + t_0)(2 t_1 - m), X_g = (m + t_0)(2 t_2 - m)

(f < g the other two axes): integer keys, the position times m^2 / 2 in the
frame of the cube-in-cube, so coincident nodes of different blocks have equal
keys exactly.

Layout of a multi-block cell-wise vector: blocks in order, each block's n^3
cells lexicographic (x fastest), (k+1)^3 local values per cell (x fastest).
"""
import numpy as np
import scipy.sparse as sp

# (kind, axis, sign, perm, flips): kind 0 centre, 1 cap
BLOCKS = [
    (0, 0, 0, (0, 1, 2), (0, 0, 0)),
    (1, 0, +1, (0, 1, 2), (0, 0, 0)),
    (1, 0, -1, (1, 0, 2), (0, 1, 0)),
    (1, 1, +1, (2, 0, 1), (0, 0, 1)),
    (1, 1, -1, (0, 2, 1), (1, 0, 0)),
    (1, 2, +1, (1, 2, 0), (0, 1, 1)),
    (1, 2, -1, (2, 1, 0), (1, 1, 0)),
]


def block_keys(b, lat, m):
    """Integer position keys (..., 3) of block-b lattice points lat (..., 3) in [0, m]."""
    kind, e, s, perm, flips = BLOCKS[b]
    lat = np.asarray(lat, dtype=np.int64)
    t = np.stack([np.where(flips[d], m - lat[..., perm[d]], lat[..., perm[d]]) for d in range(3)], axis=-1)
    if kind == 0:
        return (2 * t - m) * m
    f, g = [a for a in range(3) if a != e]
    out = np.empty_like(t)
    rad = m + t[..., 0]
    out[..., e] = s * rad * m
    out[..., f] = rad * (2 * t[..., 1] - m)
    out[..., g] = rad * (2 * t[..., 2] - m)
    return out


class MultiBlockMesh:
    def __init__(self, k, n):
        self.k, self.n, self.K = k, n, k + 1
        K, m = self.K, k * n
        self.m = m
        self.n_blocks = len(BLOCKS)
        self.cells_per_block = n ** 3
        self.local_len = K ** 3
        self.block_len = self.cells_per_block * self.local_len
        self.len = self.n_blocks * self.block_len
        e = np.arange(n ** 3)
        cc = np.stack([e % n, (e // n) % n, e // (n * n)], axis=1)
        i = np.arange(K ** 3)
        lc = np.stack([i % K, (i // K) % K, i // (K * K)], axis=1)
        lat = k * cc[:, None, :] + lc[None, :, :]                 # (cells, K^3, 3)
        keys = np.concatenate([block_keys(b, lat, m).reshape(-1, 3) for b in range(self.n_blocks)])
        self.keys, inv = np.unique(keys, axis=0, return_inverse=True)
        self.copy_node = inv.ravel()
        self.n_nodes = len(self.keys)
        self.G = sp.csr_matrix((np.ones(self.len), (np.arange(self.len), self.copy_node)),
                               shape=(self.len, self.n_nodes))
        self.valence = np.asarray(self.G.sum(axis=0)).ravel()
        # blocks sharing each node
        blk = np.repeat(np.arange(self.n_blocks), self.block_len)
        B = sp.csr_matrix((np.ones(self.len), (self.copy_node, blk)), shape=(self.n_nodes, self.n_blocks))
        self.node_blocks = np.asarray((B > 0).sum(axis=1)).ravel()

    def dss(self, v):
        """S v = G G^T v."""
        return self.G @ (self.G.T @ v)

    def dss_average(self, v):
        """S_bar v = G (G^T G)^{-1} G^T v."""
        return self.G @ ((self.G.T @ v) / self.valence)

    def expected_node_count(self):
        """Nodes of the cube-in-cube lattice: the inner (m+1)^3 cube and m shells of
        6 m^2 + 2 surface nodes each."""
        m = self.m
        return (m + 1) ** 3 + m * (6 * m * m + 2)
