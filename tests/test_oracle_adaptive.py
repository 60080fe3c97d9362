"""Pins of the adaptive-hierarchy oracle (Sec. 3.2): the refinement tree, the
hanging-node constrained active space, and the classical local multigrid of
Algorithms 4-5 with explicit level operators, edge sets and transfers.
Every pin checks the oracle against mathematics it must satisfy, not against
itself: balance and nesting of the tree, polynomial reproduction through the
constraints, exact energies, the uniform special case (where local multigrid
is the already-pinned uniform V-cycle), symmetry and positivity of the
preconditioner, continuity of its output across hanging interfaces (the
corollary on the full iteration), and convergence of the stationary
iteration to the exact constrained solution."""
import numpy as np
import pytest

from oracle.adaptive import (FEATURE_POINT, FEATURE_SPHERE, ActiveSystem, LevelSpace, LocalMultigrid,
                             RefinementTree, load_vector_level_layout)
from oracle.mesh import StructuredMesh
from oracle.multigrid import Hierarchy, make_jacobi_smoother, vcycle
from oracle.operators import interior_indices
from synthetic_inputs import uniform

TREES = {
    "point": dict(global_refinements=1, adaptive_refinements=2, feature=FEATURE_POINT,
                  center=(0.25, 0.25, 0.25), radius=0.3125, band=1.5),
    "sphere": dict(global_refinements=1, adaptive_refinements=2, feature=FEATURE_SPHERE,
                   center=(0.5, 0.5, 0.5), radius=0.3125, band=1.0),
}


def active_mask(mg):
    m = np.zeros(mg.offsets[-1])
    for l, s in enumerate(mg.spaces):
        blk = np.zeros((s.n_cells, mg.K ** 3))
        blk[mg.tree.active(l)] = 1.0
        m[mg.offsets[l]:mg.offsets[l + 1]] = blk.ravel()
    return m


@pytest.mark.parametrize("name", sorted(TREES))
def test_tree_is_nested_balanced_and_canonically_ordered(name):
    T = RefinementTree(**TREES[name])
    assert T.check_balance()
    for l in range(1, T.L + 1):
        par = T.coords[l - 1][T.refined[l - 1]]
        # children of the refined cells, 8 per parent, in child order
        assert T.n_cells(l) == 8 * len(par)
        assert np.array_equal(T.coords[l][::8] // 2, par)
        assert np.array_equal(T.coords[l].reshape(-1, 8, 3) - 2 * par[:, None, :],
                              np.broadcast_to([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)],
                                              (len(par), 8, 3)))
    # the leaves tile the cube: total active volume 1
    vol = sum(int(T.active(l).sum()) * 0.125 ** l for l in range(T.L + 1))
    assert vol == 1.0
    assert not T.refined[T.L].any()


def test_balance_pass_refines_what_the_feature_alone_leaves_unbalanced():
    """Near a sphere surface the feature marks cells whose neighbours were never
    refined; the balance pass refines those neighbours' parents, and afterwards
    every refined cell has all 26 level neighbours (2:1 across faces, edges and
    vertices)."""
    T = RefinementTree(global_refinements=1, adaptive_refinements=3, feature=FEATURE_SPHERE,
                       center=(0.3125, 0.4375, 0.5), radius=0.3125, band=0.5)
    assert T.balance_added > 0
    assert T.check_balance()


CASES = [("point", 1), ("point", 2), ("point", 3), ("sphere", 1), ("sphere", 2)]


def free_values(S, z_copies):
    """Values at the free nodes read from one copy each (for continuity checks)."""
    _, first = np.unique(S.copy_node.ravel(), return_index=True)
    return np.asarray(z_copies)[first][S.free]


@pytest.mark.parametrize("name,k", CASES)
def test_constrained_space_reproduces_polynomials_and_energies(name, k):
    """Q_k on every active cell contains x^a y^b z^c (a, b, c <= k); a function of
    that form given at the free nodes must come out exactly at every copy,
    hanging ones included (so C_HN is the interpolation of the coarse side).  With
    free boundary, A 1 = 0 and u = g.x has energy |g|^2 (unit cube)."""
    T = RefinementTree(**TREES[name])
    S = ActiveSystem(T, k, dirichlet=False)
    assert S.hanging.any()
    x = S.node_pos
    f = lambda p: p[:, 0] ** k * p[:, 1] - 0.7 * p[:, 2] ** min(k, 2) + p[:, 0] * p[:, 1] * p[:, 2] ** (k - 1)
    copies = S.G @ f(x[S.free])
    assert np.max(np.abs(copies - f(x[S.copy_node.ravel()]))) < 1e-13
    assert np.max(np.abs(S.A @ np.ones(len(S.free)))) < 1e-12
    g = np.array([0.3, -0.5, 0.8])
    u = x[S.free] @ g
    assert abs(u @ (S.A @ u) - g @ g) < 1e-12
    D = ActiveSystem(T, k, dirichlet=True)
    assert abs(D.A - D.A.T).max() < 1e-13
    if D.A.shape[0] <= 3000:
        assert np.linalg.eigvalsh(D.A.toarray()).min() > 0


@pytest.mark.parametrize("name", sorted(TREES))
def test_edge_sets_are_the_boundary_of_each_level_region(name):
    """E_l: level nodes inside the cube on the boundary of the region covered by
    level-l cells.  A uniform level has none; the interior count of a level whose
    region is a box of b cells per side (with one face on the cube boundary per
    axis) is (k b - 1)^3 and its edge count (k b)^3 - (k b - 1)^3."""
    T = RefinementTree(**TREES[name])
    k = 2
    for l in range(T.L + 1):
        s = LevelSpace(T, l, k)
        if T.n_cells(l) == 8 ** l:
            assert not s.edge.any()
        else:
            assert s.edge.any()
            assert not np.any(s.edge & s.boundary)
    if name == "point":
        s = LevelSpace(T, 3, k)           # the level-3 region is [0, 1/2]^3: 4 cells per side
        assert s.interior.sum() == (k * 4 - 1) ** 3 and s.edge.sum() == (k * 4) ** 3 - (k * 4 - 1) ** 3


def test_local_multigrid_on_a_uniform_tree_is_the_uniform_vcycle():
    """With no local refinement E_l is empty and the level distribution puts the
    whole residual on the finest level: Algorithm 5 is Algorithm 1 (the uniform
    oracle V-cycle, pinned separately), in the tree's cell order."""
    k = 2
    T = RefinementTree(global_refinements=2, adaptive_refinements=0)
    mg = LocalMultigrid(T, k, omega=0.7, nu_pre=1, nu_post=1)
    m = StructuredMesh(3, k, 4)
    h = Hierarchy(3, k, 4)
    r_cell = uniform(m.n_cellwise, seed=71).reshape(m.n_cells, -1)
    cc = m.cell_coords()
    perm = np.array([int(c[0] + 4 * c[1] + 16 * c[2]) for c in T.coords[2]])   # tree order -> structured
    rl = np.zeros(mg.offsets[-1])
    rl[mg.offsets[2]:] = r_cell[perm].ravel()
    z = mg.precondition(rl)[mg.offsets[2]:].reshape(-1, m.n_local)
    I = interior_indices(m)
    zi = vcycle(h, m.assemble(r_cell)[I], make_jacobi_smoother(0.7, 1, 1))
    zg = np.zeros(m.n_global)
    zg[I] = zi
    assert np.max(np.abs(z - m.gather(zg)[perm])) < 1e-13 * np.max(np.abs(zi))
    assert cc.shape[0] == T.n_cells(2)


@pytest.mark.parametrize("name,k", [c for c in CASES if c[1] >= 2])
def test_local_multigrid_is_symmetric_positive_and_continuous(name, k):
    """nu_pre = nu_post Jacobi sweeps make the V-cycle a symmetric operator on dual
    vectors, <r1, MG r2> = <r2, MG r1>, positive on the active space; its output on
    the active copies lies in the constrained space (the corollary on the full
    iteration: the reassembled correction satisfies the hanging-node constraints)."""
    T = RefinementTree(**TREES[name])
    mg = LocalMultigrid(T, k, omega=0.7, nu_pre=1, nu_post=1)
    S = ActiveSystem(T, k, dirichlet=True)
    am = active_mask(mg)
    r1 = uniform(mg.offsets[-1], seed=72) * am
    r2 = uniform(mg.offsets[-1], seed=73) * am
    z1, z2 = mg.precondition(r1), mg.precondition(r2)
    assert abs(r1 @ z2 - r2 @ z1) < 1e-12 * abs(r1 @ z2)
    assert r1 @ z1 > 0 and r2 @ z2 > 0
    assert np.all(z1[am == 0] == 0)
    zc = S.from_level_layout(z1, mg.spaces)
    assert np.max(np.abs(S.G @ free_values(S, zc) - zc)) < 1e-12 * np.max(np.abs(zc))


@pytest.mark.parametrize("name", sorted(TREES))
def test_stationary_local_multigrid_converges_to_the_constrained_solution(name):
    """x <- x + MG(b - A x) over the active mesh converges to the exact solution of
    C^T A C u = C^T b (the fixed point is the discrete solution), at a rate well
    below one."""
    k = 2
    T = RefinementTree(**TREES[name])
    mg = LocalMultigrid(T, k)
    S = ActiveSystem(T, k, dirichlet=True)
    b = load_vector_level_layout(T, mg.spaces, k)
    bc = S.from_level_layout(b, mg.spaces)
    uex = S.solve(bc)
    x = np.zeros(mg.offsets[-1])
    errs = []
    for _ in range(25):
        r = S.to_level_layout(bc - S.A_cells @ S.from_level_layout(x, mg.spaces), mg.spaces)
        x = x + mg.precondition(r)
        errs.append(np.max(np.abs(S.from_level_layout(x, mg.spaces) - uex)))
    assert errs[-1] < 1e-10 * np.max(np.abs(uex))
    assert (errs[-1] / errs[9]) ** (1 / 15) < 0.5
    # and the discrete solution approximates the manufactured one
    pos = S.node_pos[S.copy_node.ravel()]
    assert np.max(np.abs(uex - np.prod(np.sin(np.pi * pos), axis=1))) < 0.05
