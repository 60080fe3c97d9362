"""GPU parity of the boundary operations against the oracle: G, G^T, DSS, apply, patch inverse.

Tolerances: index maps and integer-valued sums bit-exact; FP64 arithmetic
norm-wise relative 1e-12; FP32 arithmetic norm-wise relative 1e-5 against
the FP64 oracle, ||y32 - y64|| / ||y64||.
"""
import numpy as np
import pytest
import torch

from oracle.mesh import StructuredMesh
from oracle.operators import (apply_cellwise, apply_dirichlet, assemble_csr, dss_average, dss_sum,
                              element_matrix_cartesian)
from oracle.patch import patch_inverse_cellwise
from synthetic_inputs import integer_valued, uniform

pytestmark = pytest.mark.gpu

# (dim, k, n): C1 is 2D Q2 16^2; the 3D cases span several blocks with ragged tails
CASES = [(2, 2, 16), (2, 1, 5), (2, 5, 3), (3, 1, 5), (3, 2, 3), (3, 3, 4), (3, 3, 5), (3, 4, 3), (3, 7, 2),
         (3, 8, 2), (2, 3, 1), (3, 3, 1), (3, 7, 1)]   # n = 1: a single cell, every node on the boundary


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("dim,k,n", CASES)
def test_gather_assemble_bit_exact(gpu_lib, dim, k, n):
    fe = gpu_lib
    m = StructuredMesh(dim, k, n)
    P = fe.Problem(dim, k, n, bc=0)
    xg = uniform(m.n_global, seed=100)
    xc = P.cellvec()
    P.gather(dev(xg), xc)
    assert np.array_equal(host(xc), m.gather(xg).ravel())
    v = integer_valued(m.n_cellwise, seed=101)
    yg = torch.zeros(m.n_global, dtype=torch.float64, device="cuda")
    P.assemble(dev(v), yg)
    assert np.array_equal(host(yg), m.assemble(v))


@pytest.mark.parametrize("dim,k,n", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_assembled_norm2_exact_on_integers(gpu_lib, dim, k, n, dtype):
    """||G^T v||^2 (Sec. 2.1: G^T sums the cell copies): on integer-valued copies
    every sum and square is exact, so the value is the oracle's to the bit; each
    node counted once, whichever copy counts it."""
    fe = gpu_lib
    m = StructuredMesh(dim, k, n)
    P = fe.Problem(dim, k, n, bc=0)
    v = integer_valued(m.n_cellwise, seed=103)
    expect = float(np.sum(m.assemble(v) ** 2))
    assert P.assembled_norm2(dev(v, dtype)) == expect


@pytest.mark.parametrize("dim,k,n", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_dss_bit_exact_on_integers(gpu_lib, dim, k, n, dtype):
    fe = gpu_lib
    m = StructuredMesh(dim, k, n)
    P = fe.Problem(dim, k, n, bc=0)
    v = integer_valued(m.n_cellwise, seed=102)
    for averaging in (False, True):
        t = dev(v, dtype)
        P.dss(t, averaging=averaging)
        expect = (dss_average if averaging else dss_sum)(m, v.reshape(m.n_cells, m.n_local)).ravel()
        assert np.array_equal(host(t), expect)


@pytest.mark.parametrize("dim,k,n", [(2, 2, 16), (3, 3, 4), (3, 7, 2)])
def test_dss_random_and_projection(gpu_lib, dim, k, n):
    fe = gpu_lib
    m = StructuredMesh(dim, k, n)
    P = fe.Problem(dim, k, n, bc=0)
    v = uniform(m.n_cellwise, seed=103)
    t = dev(v)
    P.dss(t)
    assert relerr(host(t), dss_sum(m, v.reshape(m.n_cells, -1)).ravel()) < 1e-15
    # S_bar G x = G x bit-exactly (pairwise cascade of identical copies, power-of-two valence)
    x = m.gather(uniform(m.n_global, seed=104)).ravel()
    t = dev(x)
    P.dss(t, averaging=True)
    assert np.array_equal(host(t), x)


@pytest.mark.parametrize("dim,k,n", CASES)
@pytest.mark.parametrize("bc", [0, 1])
def test_apply_fp64_and_fp32(gpu_lib, dim, k, n, bc):
    fe = gpu_lib
    m = StructuredMesh(dim, k, n)
    E = element_matrix_cartesian(dim, k, m.h)
    P = fe.Problem(dim, k, n, bc=bc)
    x = m.gather(uniform(m.n_global, seed=105)).ravel()
    expect = (apply_dirichlet if bc else apply_cellwise)(m, E, x).ravel()
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        y = P.cellvec(dtype)
        P.apply(dev(x, dtype), y)
        assert relerr(host(y), expect) < tol, (dtype, relerr(host(y), expect))
    # assembled result equals the CSR product (bc = 0)
    if bc == 0:
        y = P.cellvec()
        P.apply(dev(x), y)
        A = assemble_csr(m, E)
        xg = uniform(m.n_global, seed=105)
        assert relerr(m.assemble(host(y)), A @ xg) < 1e-12


@pytest.mark.parametrize("k,n", [(3, 15), (3, 16), (3, 17), (3, 23), (3, 33), (7, 5), (2, 17)])
def test_apply_block_seams(gpu_lib, k, n):
    """Sizes that place the apply's per-block cell runs across x-row boundaries
    differently (Q3: 16 cells per pass, two passes per block in FP32; fewer cells
    per row than per pass, exactly one row, one more, several rows and a ragged
    last block), every entry against the dense per-cell oracle in both
    precisions."""
    fe = gpu_lib
    m = StructuredMesh(3, k, n)
    E = element_matrix_cartesian(3, k, m.h)
    P = fe.Problem(3, k, n, bc=1)
    x = m.gather(uniform(m.n_global, seed=108)).ravel()
    expect = apply_dirichlet(m, E, x).ravel()
    for dtype, tol, ent in ((torch.float64, 1e-12, 1e-11), (torch.float32, 1e-5, 1e-4)):
        y = P.cellvec(dtype)
        P.apply(dev(x, dtype), y)
        got = host(y)
        assert relerr(got, expect) < tol, (dtype, relerr(got, expect))
        assert np.max(np.abs(got - expect)) <= ent * np.max(np.abs(expect)), dtype
    P.close()


@pytest.mark.parametrize("dim,k,n", [(2, 2, 16), (2, 3, 5), (3, 1, 4), (3, 2, 3), (3, 3, 4), (3, 3, 5),
                                     (3, 2, 9), (3, 3, 8), (3, 3, 1), (3, 4, 3), (3, 5, 3), (3, 6, 3),
                                     (3, 7, 3), (3, 8, 2)])
def test_patch_inverse_fp64_fp32_and_continuity(gpu_lib, dim, k, n):
    fe = gpu_lib
    m = StructuredMesh(dim, k, n)
    A = assemble_csr(m, element_matrix_cartesian(dim, k, m.h))
    P = fe.Problem(dim, k, n, bc=1)
    r = uniform(m.n_cellwise, seed=106)
    expect = patch_inverse_cellwise(A, m, r.reshape(m.n_cells, -1), shared=True).ravel()
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        z = P.cellvec(dtype)
        P.patch_inverse(dev(r, dtype), z)
        zh = host(z)
        assert relerr(zh, expect) < tol, (dtype, relerr(zh, expect))
        # every copy of a node holds bit-identical values
        idx = m.global_index_map().ravel()
        first = np.full(m.n_global, np.nan)
        first[idx[::-1]] = zh[::-1]
        assert np.array_equal(zh, first[idx])


def test_apply_rejects_bad_arguments(gpu_lib):
    fe = gpu_lib
    P = fe.Problem(3, 2, 2)
    x = P.cellvec()
    with pytest.raises(fe.FeError) as e:
        P.apply(x, x)
    assert e.value.status == -1
    with pytest.raises(fe.FeError):
        fe.Problem(3, 9, 2)
    with pytest.raises(fe.FeError):
        P.patch_inverse(x, P.cellvec(), factors=1)
