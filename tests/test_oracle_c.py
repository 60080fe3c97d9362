"""The C oracle (oracle/csrc/fe_oracle.c, used for the CPU baseline at full
benchmark sizes) against the numpy oracle's definitions: the cell-wise
Dirichlet apply (dense A_K per cell, boundary copies masked) and the vertex-patch
inverse, the latter also against the per-patch dense solves on the assembled
matrix (one Cholesky per patch), on meshes with no patch, one patch, and
several tiles of patches, k = 1, 2, 3, 7.
"""
import numpy as np
import pytest

from oracle import c_oracle
from oracle.mesh import StructuredMesh
from oracle.operators import apply_dirichlet, assemble_csr, element_matrix_cartesian
from oracle.patch import patch_inverse_cartesian, patch_inverse_cellwise
from synthetic_inputs import uniform


@pytest.fixture(scope="module", autouse=True)
def built():
    c_oracle.build()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("k,n", [(1, 1), (1, 4), (2, 3), (3, 1), (3, 2), (3, 5), (7, 2)])
def test_c_apply_matches_numpy_oracle(k, n):
    m = StructuredMesh(3, k, n)
    E = element_matrix_cartesian(3, k, m.h)
    x = uniform(m.n_cellwise, seed=11)
    expect = apply_dirichlet(m, E, x).ravel()
    got = c_oracle.CartesianOracle(m).apply_dirichlet(x)
    assert rel(got, expect) < 1e-13


@pytest.mark.parametrize("k,n", [(1, 1), (1, 4), (2, 3), (3, 1), (3, 2), (3, 5), (7, 2)])
def test_c_patch_inverse_matches_numpy_oracle(k, n):
    m = StructuredMesh(3, k, n)
    r = uniform(m.n_cellwise, seed=12)
    expect = patch_inverse_cartesian(m, r.reshape(m.n_cells, -1)).ravel()
    got = c_oracle.CartesianOracle(m).patch_inverse(r)
    if n == 1:   # no interior vertex: no patch
        assert np.all(got == 0.0) and np.all(expect == 0.0)
        return
    assert rel(got, expect) < 1e-13


@pytest.mark.parametrize("k,n", [(2, 3), (3, 3)])
def test_c_patch_inverse_matches_per_patch_solves(k, n):
    m = StructuredMesh(3, k, n)
    A = assemble_csr(m, element_matrix_cartesian(3, k, m.h))
    r = uniform(m.n_cellwise, seed=13)
    expect = patch_inverse_cellwise(A, m, r.reshape(m.n_cells, -1)).ravel()
    got = c_oracle.CartesianOracle(m).patch_inverse(r)
    assert rel(got, expect) < 1e-12


def test_c_patch_inverse_copies_identical():
    """Every cell-wise copy of a node carries the same value (z = G zg)."""
    m = StructuredMesh(3, 3, 4)
    z = c_oracle.CartesianOracle(m).patch_inverse(uniform(m.n_cellwise, seed=14))
    idx = m.global_index_map().ravel()
    first = np.full(m.n_global, np.nan)
    first[idx[::-1]] = z[::-1]
    assert np.array_equal(z, first[idx])
