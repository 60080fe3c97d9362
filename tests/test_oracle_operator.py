"""Pins for the oracle's mesh, operator and DSS against closed forms and invariants."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.kron import KroneckerOperator, global_1d
from oracle.mesh import StructuredMesh
from oracle.operators import (apply_cellwise, assemble_csr, dirichlet_block, dss_average,
                              dss_sum, element_matrix_cartesian)
from oracle.basis import gll_nodes
from synthetic_inputs import integer_valued, uniform


def node_coords(mesh):
    """Physical coordinates of the global nodes, (n_global, d)."""
    xi = gll_nodes(mesh.k)
    line = np.empty(mesh.N)
    for e in range(mesh.n):
        line[mesh.k * e:mesh.k * e + mesh.k + 1] = (e + xi) / mesh.n
    gc = mesh.global_coords()
    return line[gc]


@pytest.mark.parametrize("dim,k,n", [(2, 1, 3), (2, 2, 4), (3, 1, 2), (3, 3, 2), (3, 2, 3)])
def test_gather_valence_closed_form(dim, k, n):
    m = StructuredMesh(dim, k, n)
    G = m.gather_matrix()
    kappa = np.asarray((G.T @ G).diagonal()).ravel()
    gc = m.global_coords()
    shared = (gc % k == 0) & (gc > 0) & (gc < k * n)
    assert np.array_equal(kappa, np.prod(1 + shared, axis=1))
    # G^T G is diagonal
    GtG = (G.T @ G).tocoo()
    assert np.all(GtG.row == GtG.col)


@pytest.mark.parametrize("dim,k,n", [(2, 2, 3), (3, 3, 2)])
def test_dss_brute_force_on_integers(dim, k, n):
    """S v = G G^T v: every copy becomes the sum of all copies (exact on integers)."""
    m = StructuredMesh(dim, k, n)
    v = integer_valued(m.n_cellwise, seed=5).reshape(m.n_cells, m.n_local)
    idx = m.global_index_map()
    expect = np.empty_like(v)
    for e in range(m.n_cells):
        for i in range(m.n_local):
            expect[e, i] = v[idx == idx[e, i]].sum()
    assert np.array_equal(dss_sum(m, v), expect)
    kappa = m.valence_global()[idx]
    assert np.array_equal(dss_average(m, v), expect / kappa)


def test_averaging_dss_is_projection_and_valence_baking():
    m = StructuredMesh(3, 2, 3)
    xg = uniform(m.n_global, seed=3)
    x = m.gather(xg)
    # S_bar G x = G x (the oracle sums copies sequentially, so only to rounding)
    assert np.max(np.abs(dss_average(m, x) - x)) < 4e-16
    # eq. valence_baking: S_bar K_cell D_cell^{-1} v = D_cell^{-1} S v
    d_cell = m.gather(uniform(m.n_global, seed=4, low=1.0, high=2.0))
    kappa_cell = m.gather(m.valence_global())
    v = uniform(m.n_cellwise, seed=6).reshape(x.shape)
    lhs = dss_average(m, kappa_cell * v / d_cell)
    rhs = dss_sum(m, v) / d_cell
    assert np.max(np.abs(lhs - rhs)) < 1e-14


@pytest.mark.parametrize("dim,k,n", [(2, 2, 4), (3, 1, 3), (3, 3, 2), (3, 4, 2)])
def test_operator_kills_constants_and_is_symmetric(dim, k, n):
    m = StructuredMesh(dim, k, n)
    A = assemble_csr(m, element_matrix_cartesian(dim, k, m.h))
    assert np.max(np.abs(A @ np.ones(m.n_global))) < 1e-12
    assert abs(A - A.T).max() < 1e-13
    AII = dirichlet_block(A, m).toarray()
    sla.cholesky(AII)                                      # SPD


@pytest.mark.parametrize("dim,k,n", [(2, 2, 3), (3, 2, 2), (3, 3, 2), (2, 5, 2)])
def test_energy_of_polynomials(dim, k, n):
    """a(u,u) = int |grad u|^2 exactly for u = x^2 (=4/3) and linear u = g.x (=|g|^2)."""
    m = StructuredMesh(dim, k, n)
    A = assemble_csr(m, element_matrix_cartesian(dim, k, m.h))
    X = node_coords(m)
    u = X[:, 0] ** 2
    assert abs(u @ A @ u - 4.0 / 3.0) < 1e-12
    g = np.array([0.3, -1.1, 0.7][:dim])
    u = X @ g
    assert abs(u @ A @ u - g @ g) < 1e-12
    # mixed monomial in 2D/3D: u = x*y, int |grad u|^2 = int y^2 + x^2 = 2/3
    u = X[:, 0] * X[:, 1]
    assert abs(u @ A @ u - 2.0 / 3.0) < 1e-12


def test_q1_eigenvalues_closed_form():
    """Q1 1D Dirichlet: lambda_j = 6 h^-2 (1 - cos(j pi h)) / (2 + cos(j pi h))."""
    n = 17
    K1, M1 = global_1d(1, n)
    lam = sla.eigh(K1, M1, eigvals_only=True)
    h = 1.0 / n
    j = np.arange(1, n)
    exact = np.sort(6 / h ** 2 * (1 - np.cos(j * np.pi * h)) / (2 + np.cos(j * np.pi * h)))
    assert np.max(np.abs(lam - exact) / exact) < 1e-12


def test_smallest_eigenvalue_converges_to_3pi2():
    for (k, n, tol) in [(3, 64, 1e-10), (2, 16, 5e-6)]:
        ko = KroneckerOperator(3, k, n)
        rel = abs(ko.min_eigenvalue() - 3 * np.pi ** 2) / (3 * np.pi ** 2)
        assert rel < tol


@pytest.mark.parametrize("dim,k,n", [(2, 2, 4), (3, 3, 3), (3, 2, 4)])
def test_kronecker_oracle_matches_csr(dim, k, n):
    """Two independent constructions of A_II: CSR from element matrices and 1D Kronecker sums."""
    m = StructuredMesh(dim, k, n)
    AII = dirichlet_block(assemble_csr(m, element_matrix_cartesian(dim, k, m.h)), m)
    ko = KroneckerOperator(dim, k, n)
    x = uniform(AII.shape[0], seed=1)
    assert np.max(np.abs(AII @ x - ko.apply(x))) < 1e-12 * np.abs(AII @ x).max()
    b = uniform(AII.shape[0], seed=2)
    xs = ko.solve(b)
    assert np.linalg.norm(AII @ xs - b) < 1e-11 * np.linalg.norm(b)
    # generalized eigenvalues of the 3D problem are sums of the 1D ones
    if dim == 2:
        Md = np.kron(ko.M1, ko.M1)
        lam = sla.eigh(AII.toarray(), Md, eigvals_only=True)
        expect = np.sort((ko.lam[:, None] + ko.lam[None, :]).ravel())
        assert np.max(np.abs(lam - expect) / expect) < 1e-10


def test_cellwise_apply_assembles_to_csr():
    m = StructuredMesh(3, 3, 3)
    E = element_matrix_cartesian(3, 3, m.h)
    xg = uniform(m.n_global, seed=0)
    y = apply_cellwise(m, E, m.gather(xg))
    A = assemble_csr(m, E)
    assert np.max(np.abs(m.assemble(y) - A @ xg)) < 1e-13


@pytest.mark.parametrize("dim,k,ns,rate_min", [(2, 2, (4, 8, 16), 2.8), (3, 3, (2, 4, 8), 3.7)])
def test_manufactured_solution_converges_at_order_k_plus_1(dim, k, ns, rate_min):
    from oracle.rhs import l2_error_cartesian, load_vector_cartesian
    errs = []
    for n in ns:
        m = StructuredMesh(dim, k, n)
        ko = KroneckerOperator(dim, k, n)
        b = m.assemble(load_vector_cartesian(m))
        bmask = m.boundary_mask_global()
        u = np.zeros(m.n_global)
        u[~bmask] = ko.solve(b[~bmask])
        errs.append(l2_error_cartesian(m, m.gather(u)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > rate_min), (errs, rates)
