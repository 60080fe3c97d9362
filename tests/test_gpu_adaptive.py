"""GPU parity of adaptive local smoothing (Sec. 3.2, Algorithms 4-5; Sec. 4.3;
Sec. 5) against the oracle's classical local multigrid with explicit level
operators, edge sets, transfers and hanging-node constraints: the refinement
tree and brick tables (bit-exact), the refinement edge found by one DSS
(bit-exact), the structured cascade on the level meshes (bit-exact on
integer data where every copy has its partner), the masked inverse
diagonal, the transfers, the operator and load vector, the V-cycle (the
theorem on the equivalence with classical local multigrid), and CG on the
active mesh (the exact constrained solution; iteration counts flat in the
adaptive depth, Sec. 6.3)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle.adaptive import (FEATURE_POINT, FEATURE_SPHERE, ActiveSystem, LevelSpace, LocalMultigrid,
                             RefinementTree, load_vector_level_layout, prolongation)
from oracle.operators import element_matrix_cartesian
from synthetic_inputs import integer_valued, uniform

pytestmark = pytest.mark.gpu
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_convergence.json")))

TREES = {
    "point": dict(global_refinements=1, adaptive_refinements=2, feature=FEATURE_POINT,
                  center=(0.25, 0.25, 0.25), radius=0.3125, band=1.5),
    "sphere": dict(global_refinements=1, adaptive_refinements=2, feature=FEATURE_SPHERE,
                   center=(0.5, 0.5, 0.5), radius=0.3125, band=1.0),
    "sphere_off": dict(global_refinements=1, adaptive_refinements=3, feature=FEATURE_SPHERE,
                       center=(0.3125, 0.4375, 0.5), radius=0.3125, band=0.5),
}


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def make(fe, name, k):
    spec = TREES[name]
    return fe.Adaptive(k, spec["global_refinements"], spec["adaptive_refinements"], spec["feature"],
                       spec["center"], spec["radius"], spec["band"]), RefinementTree(**spec)


def jacobi_opts(fe, **kw):
    o = dict(smoother=fe.SMOOTH_JACOBI, inner=fe.F64, omega=0.7, nu_pre=1, nu_post=1)
    o.update(kw)
    return fe.default_opts(**o)


@pytest.mark.parametrize("name", sorted(TREES))
def test_tree_and_brick_tables_match_the_oracle(gpu_lib, name):
    fe = gpu_lib
    print("adaptive tree", name, flush=True)
    A, T = make(fe, name, 2)
    assert A.n_levels == T.L + 1
    assert A.active_cells == sum(int(T.active(l).sum()) for l in range(T.L + 1))
    for l in range(T.L + 1):
        coords, refined = A.level_info(l)
        assert np.array_equal(coords, T.coords[l]) and np.array_equal(refined, T.refined[l])
        if l == 0:
            continue
        nbr, par = A.brick_neighbors(l)
        assert np.array_equal(par, np.flatnonzero(T.refined[l - 1]))
        pc = T.coords[l - 1][par]
        brick_of = {tuple(c): b for b, c in enumerate(pc)}
        for b, c in enumerate(pc):
            for a in range(3):
                for sgn in (0, 1):
                    q = c.copy()
                    q[a] += 1 if sgn else -1
                    assert nbr[b, 2 * a + sgn] == brick_of.get(tuple(q), -1)
    A.close()


@pytest.mark.parametrize("name", sorted(TREES))
@pytest.mark.parametrize("k", [2, 3])
def test_edge_mask_dss_and_dinv_match_the_oracle(gpu_lib, name, k):
    """E_l from one DSS of the face marker equals the geometric refinement edge on
    every copy inside the cube; the cascade sums every copy of an interior node
    exactly (integer data); the masked, valence-baked inverse diagonal is
    kappa / diag(A_l) on S_l and 0 on E_l and the boundary."""
    fe = gpu_lib
    print("adaptive edge/dss/dinv", name, k, flush=True)
    A, T = make(fe, name, k)
    for l in range(T.L + 1):
        s = LevelSpace(T, l, k)
        bnd = s.boundary[s.copy_node].ravel()
        edge = s.edge[s.copy_node].ravel()
        inter = s.interior[s.copy_node].ravel()
        m = host(A.edge_mask(l))
        assert np.array_equal(m[~bnd] > 0, edge[~bnd]), l
        # DSS sum / average on the interior copies (every copy has its partner)
        v = integer_valued(A.offsets[l + 1] - A.offsets[l], seed=80 + l)
        vd = dev(v)
        A.dss(l, vd)
        expect = (s.G @ (s.G.T @ v))
        assert np.array_equal(host(vd)[inter], expect[inter])
        va = dev(v)
        A.dss(l, va, averaging=True)
        kap = np.asarray(s.G.sum(axis=0)).ravel()[s.copy_node].ravel()
        assert np.array_equal(host(va)[inter], expect[inter] / kap[inter])
        if l == 0:
            continue
        dinv = host(A.dinv(l))
        ref = np.where(inter, kap / s.diag[s.copy_node].ravel(), 0.0)
        assert np.max(np.abs(dinv - ref)) <= 1e-14 * np.max(np.abs(ref))
    A.close()


@pytest.mark.parametrize("name", sorted(TREES))
def test_transfers_apply_and_load_vector_match_the_oracle(gpu_lib, name):
    """Algorithm 2: the cell-wise prolongation of a continuous coarse field is the
    gather of P_CG u (lemma on commutativity); Algorithm 3: the assembled
    restriction of an unassembled residual is P_CG^T of the assembled residual
    (lemma on unassembled restriction); the operator is A_K per active cell and the
    load vector the oracle's quadrature."""
    fe = gpu_lib
    k = 3
    print("adaptive transfers/apply/rhs", name, flush=True)
    A, T = make(fe, name, k)
    spaces = [LevelSpace(T, l, k) for l in range(T.L + 1)]
    for l in range(1, T.L + 1):
        c, f = spaces[l - 1], spaces[l]
        P = prolongation(T, c, f)
        uc = uniform(c.n_nodes, seed=90 + l)
        ef = A.level_vec(l)
        A.prolongate_add(l, dev(c.G @ uc), ef)
        assert np.max(np.abs(host(ef) - f.G @ (P @ uc))) < 1e-13 * np.max(np.abs(uc))
        r = uniform(f.n_cells * (k + 1) ** 3, seed=95 + l)
        bc = A.level_vec(l - 1)
        A.restrict_add(l, dev(r), A.level_vec(l), bc)
        got = c.G.T @ host(bc)
        assert np.max(np.abs(got - P.T @ (f.G.T @ r))) < 1e-12 * np.max(np.abs(r))
    # active-mesh operator and load vector
    x = np.concatenate([uniform(s.n_cells * (k + 1) ** 3, seed=99 + l).reshape(s.n_cells, -1)
                        * T.active(l)[:, None] for l, s in enumerate(spaces)], axis=None)
    y = A.vec()
    A.apply(dev(x), y)
    expect = []
    for l, s in enumerate(spaces):
        E = element_matrix_cartesian(3, k, 0.5 ** l)
        xl = x[A.offsets[l]:A.offsets[l + 1]].reshape(s.n_cells, -1)
        expect.append((xl @ E.T).ravel())
    expect = np.concatenate(expect)
    assert np.max(np.abs(host(y) - expect)) < 1e-13 * np.max(np.abs(expect))
    b = A.vec()
    A.rhs_manufactured(b)
    ref = load_vector_level_layout(T, spaces, k)
    assert np.max(np.abs(host(b) - ref)) < 1e-13 * np.max(np.abs(ref))
    A.close()


@pytest.mark.parametrize("name", sorted(TREES))
@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("nu", [1, 2])
def test_local_vcycle_equals_classical_local_multigrid(gpu_lib, name, k, nu):
    """The theorem on the equivalence of cell-wise and classical local multigrid:
    Algorithm 4 on the GPU (structured cascade with masked refinement edges,
    unassembled transfers, no constraints) gives, copy by copy, the gathered
    correction of the classical local V-cycle with explicit level operators,
    frozen edge values and P_CG^T restriction."""
    fe = gpu_lib
    print("adaptive vcycle", name, k, nu, flush=True)
    A, T = make(fe, name, k)
    mg = LocalMultigrid(T, k, omega=0.7, nu_pre=nu, nu_post=nu)
    act = np.concatenate([np.repeat(T.active(l), (k + 1) ** 3) for l in range(T.L + 1)]).astype(float)
    r = uniform(A.len, seed=120 + k) * act
    z = A.vec()
    A.precondition(dev(r), z, jacobi_opts(fe, nu_pre=nu, nu_post=nu))
    ref = mg.precondition(r)
    got = host(z)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    A.close()


@pytest.mark.parametrize("name", ["point", "sphere"])
def test_adaptive_pcg_reaches_the_constrained_solution(gpu_lib, name):
    """CG on the active mesh, preconditioned by Algorithm 4, converges to the exact
    solution of the hanging-node-constrained system C^T A C u = C^T b (the oracle
    assembles C explicitly); the iterate is continuous across hanging interfaces."""
    fe = gpu_lib
    k = 2
    print("adaptive pcg", name, flush=True)
    A, T = make(fe, name, k)
    spaces = [LevelSpace(T, l, k) for l in range(T.L + 1)]
    S = ActiveSystem(T, k, dirichlet=True)
    b = A.vec()
    A.rhs_manufactured(b)
    x = A.vec()
    rep = A.pcg(b, x, jacobi_opts(fe, stop=1, tol=1e-26, maxit=100))
    assert rep["converged"], rep
    bc = S.from_level_layout(host(b), spaces)
    uex = S.solve(bc)
    got = S.from_level_layout(host(x), spaces)
    assert np.max(np.abs(got - uex)) < 1e-10 * np.max(np.abs(uex))
    A.close()


def test_adaptive_error_paths(gpu_lib):
    fe = gpu_lib
    with pytest.raises(fe.FeError):
        fe.Adaptive(6, 1, 1)
    with pytest.raises(fe.FeError):
        fe.Adaptive(2, 10, 4)
    A = fe.Adaptive(2, 1, 1)
    b = A.vec()
    with pytest.raises(fe.FeError):
        A.pcg(b, A.vec(), jacobi_opts(fe, stop=0))
    with pytest.raises(fe.FeError):
        A.pcg(b, A.vec(), fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, stop=1))
    A.close()


@pytest.mark.parametrize("k", [2, 3])
def test_iterations_are_flat_in_the_adaptive_depth(gpu_lib, k):
    """Sec. 6.3, Table mg_adaptive_iters: CG iterations to a 1e-14 reduction of the
    energy measure do not grow with the number of adaptive refinements (cube,
    global refinement 4 here, refinement toward a sphere surface)."""
    fe = gpu_lib
    its = []
    for a in (1, 2, 3):
        print("adaptive depth", k, a, flush=True)
        A = fe.Adaptive(k, 4, a, fe.FEATURE_SPHERE, (0.5, 0.5, 0.5), 0.3125, 1.0)
        b = A.vec()
        A.rhs_manufactured(b)
        x = A.vec()
        rep = A.pcg(b, x, jacobi_opts(fe, stop=1, tol=1e-14, maxit=60))
        assert rep["converged"]
        its.append(rep["iters"])
        A.close()
    gold = GOLDEN["cg_iterations_cube_adaptive"]["p%d" % k]
    print("p=%d iterations for 1, 2, 3 adaptive refinements: %s (paper: %s)" % (k, its, gold[:3]))
    assert max(its) - min(its) <= 1, its
    assert all(abs(i - g) <= 2 for i, g in zip(its, gold)), (its, gold)
