"""Pins for the deformed-geometry oracle: Cartesian limit, invariants, closed-form Jacobian."""
import numpy as np
import pytest

from oracle.geometry import DeformedGeometry
from oracle.mesh import StructuredMesh
from oracle.operators import assemble_csr, element_matrix_cartesian
from synthetic_inputs import coefficient_modes, uniform


@pytest.mark.parametrize("k,n", [(1, 3), (2, 2), (3, 2)])
def test_undeformed_constant_coefficient_is_cartesian(k, n):
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, 0.0, None)
    E = g.element_matrices()
    ref = element_matrix_cartesian(3, k, m.h)
    assert np.max(np.abs(E - ref[None])) < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("k,n", [(2, 3), (3, 2)])
def test_deformed_operator_symmetric_kills_constants_and_spd(k, n):
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, 0.1, coefficient_modes(2))
    E = g.element_matrices()
    assert np.max(np.abs(E - np.transpose(E, (0, 2, 1)))) < 1e-13 * np.abs(E).max()
    assert np.max(np.abs(E.sum(axis=2))) < 1e-12 * np.abs(E).max()
    A = assemble_csr(m, E)
    I = np.flatnonzero(~m.boundary_mask_global())
    np.linalg.cholesky(A[I][:, I].toarray())
    # matrix-free quadrature apply equals the dense element matrices
    x = m.gather(uniform(m.n_global, seed=3))
    assert np.max(np.abs(g.apply(x) - np.einsum("eij,ej->ei", E, x))) < 1e-12 * np.abs(E).max()
    assert np.allclose(g.diagonal(), np.einsum("eii->ei", E), rtol=1e-13, atol=0)


def test_coefficient_scaled_to_unit_max_exponent():
    m = StructuredMesh(3, 2, 3)
    g = DeformedGeometry(m, 0.1, coefficient_modes(7))
    lg = np.log(g.kappa)
    assert abs(np.max(np.abs(lg)) - 1.0) < 1e-14
    assert np.exp(-1) - 1e-14 <= g.kappa.min() and g.kappa.max() <= np.exp(1) + 1e-14


def test_jacobian_converges_to_closed_form():
    """det of the continuous map: 1 + 2 pi amp (c s s + s c s + s s c)."""
    amp = 0.1
    errs = []
    for n in (4, 8):
        m = StructuredMesh(3, 3, n)
        g = DeformedGeometry(m, amp, None)
        ref = np.stack(np.meshgrid(*(g.xq,) * 3, indexing="ij"), -1)   # placeholder shape
        cc = m.cell_coords()
        xq = g.xq
        pts = np.stack(np.meshgrid(xq, xq, xq, indexing="ij"), -1)[..., ::-1].reshape(-1, 3)
        xh = (cc[:, None, :] + pts[None]) / n          # reference (undeformed) point per (cell, q)
        s, c = np.sin(2 * np.pi * xh), np.cos(2 * np.pi * xh)
        det = 1 + 2 * np.pi * amp * (c[..., 0] * s[..., 1] * s[..., 2] + s[..., 0] * c[..., 1] * s[..., 2]
                                     + s[..., 0] * s[..., 1] * c[..., 2])
        errs.append(np.max(np.abs(g.detJ * n ** 3 - det)))
        assert 0.27 < (g.detJ * n ** 3).min() and (g.detJ * n ** 3).max() < 1.73
        del ref
    # derivative of the degree-k interpolant: O(h^k) asymptotically, at least a factor 4.5 here
    assert errs[1] < errs[0] / 4.5 and errs[1] < 5e-3, errs


def test_volume_and_linear_energy_converge():
    for n, tol in ((2, 2e-2), (4, 2e-3)):
        m = StructuredMesh(3, 3, n)
        g = DeformedGeometry(m, 0.1, None)
        vol = np.sum(g.W[None, :] * g.detJ)
        assert abs(vol - 1.0) < tol
        gv = np.array([0.3, -0.5, 0.8])
        u = np.einsum("ejd,d->ej", g.X, gv)       # linear physical function at the geometry nodes
        e = np.einsum("ej,ej->", u, g.apply(u))
        assert abs(e - gv @ gv) < 5 * tol


def test_averaged_separable_fit_is_exact_on_cartesian_cells():
    from oracle.patch import patch_matrices
    from oracle.sepfit import averaged_weights, design_matrix, sep_matrix
    assert np.linalg.matrix_rank(design_matrix()) == 9     # three scaling gauges per patch
    for k in (2, 3):
        m = StructuredMesh(3, k, 3)
        g = DeformedGeometry(m, 0.0, None)
        A = assemble_csr(m, g.element_matrices())
        w = averaged_weights(g)
        P = patch_matrices(A, m)
        for p in range(P.shape[0]):
            S = sep_matrix(k, w[p])
            assert np.max(np.abs(S - P[p])) < 1e-12 * np.abs(P[p]).max()


def test_averaged_separable_fit_tracks_deformed_patch():
    """On the deformed mesh the surrogate is close to, but not equal to, the patch matrix."""
    from oracle.patch import patch_matrices
    from oracle.sepfit import averaged_weights, sep_matrix
    m = StructuredMesh(3, 2, 4)
    g = DeformedGeometry(m, 0.1, coefficient_modes(5))
    A = assemble_csr(m, g.element_matrices())
    w = averaged_weights(g)
    P = patch_matrices(A, m)
    rel = [np.linalg.norm(sep_matrix(2, w[p]) - P[p]) / np.linalg.norm(P[p]) for p in range(P.shape[0])]
    assert 1e-3 < max(rel) < 0.6


def test_chunked_scale_and_cell_subset_match_whole_mesh():
    """The chunked coefficient scale equals the whole-mesh one, and the geometry of
    a cell subset (given that scale) equals the whole-mesh geometry on those cells."""
    from oracle.geometry import coefficient_scale
    m = StructuredMesh(3, 2, 3)
    coef = coefficient_modes(5)
    full = DeformedGeometry(m, 0.1, coef)
    assert coefficient_scale(m, 0.1, coef, chunk=4) == full.scale
    cells = np.array([0, 5, 13, 26])
    sub = DeformedGeometry(m, 0.1, coef, scale=full.scale, cells=cells)
    assert np.array_equal(sub.element_matrices(), full.element_matrices()[cells])
    x = uniform(len(cells) * m.n_local, seed=4).reshape(len(cells), -1)
    ref = np.einsum("eij,ej->ei", full.element_matrices()[cells], x)
    assert np.max(np.abs(sub.apply(x) - ref)) < 1e-12 * np.abs(ref).max()
    with pytest.raises(ValueError):
        DeformedGeometry(m, 0.1, coef, cells=cells)
