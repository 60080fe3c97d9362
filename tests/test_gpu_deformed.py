"""GPU parity on the deformed, variable-coefficient mesh: general operator, load vector,
averaged-geometry patch inverse and the MG-PCG solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle.geometry import DeformedGeometry
from oracle.mesh import StructuredMesh
from oracle.operators import assemble_csr, boundary_mask_cellwise
from oracle.sepfit import averaged_weights, sep_patch_inverse_cellwise
from synthetic_inputs import coefficient_modes, uniform

pytestmark = pytest.mark.gpu
AMP = 0.1


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def problem(fe, k, n, bc=1, seed=2):
    return fe.Problem(3, k, n, geometry=fe.GEOM_DEFORMED, bc=bc, deform_amp=AMP, coef=coefficient_modes(seed))


@pytest.mark.parametrize("k,n", [(1, 4), (2, 3), (3, 4), (7, 2)])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("metric", [0, 1])
def test_general_apply(gpu_lib, k, n, bc, metric):
    """metric = 0: the stored metric per Gauss point; metric = 1: the metric formed
    in the kernel from the map (only the coefficient is read)."""
    fe = gpu_lib
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, AMP, coefficient_modes(2))
    P = problem(fe, k, n, bc)
    P.set_metric_mode(metric)
    x = m.gather(uniform(m.n_global, seed=300)).ravel()
    if bc:
        mask = boundary_mask_cellwise(m).ravel()
        expect = g.apply(np.where(mask, 0.0, x)).ravel()
        expect[mask] = 0.0
    else:
        expect = g.apply(x).ravel()
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        y = P.cellvec(dtype)
        P.apply(dev(x, dtype), y)
        assert relerr(host(y), expect) < tol, (dtype, relerr(host(y), expect))
        # entry-wise: no entry off by more than the tolerance times the largest entry
        assert np.max(np.abs(host(y) - expect)) <= 10 * tol * np.max(np.abs(expect)), dtype


def test_formed_metric_solve_matches_stored_metric(gpu_lib):
    """The MG-PCG solve with the metric formed in the kernel takes the iterations of
    the stored-metric solve and reaches the same solution."""
    fe = gpu_lib
    P = problem(fe, 3, 8)
    b = P.cellvec()
    P.rhs_manufactured(b)
    opts = fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F32, flexible=1, factors=1, nu_pre=1, nu_post=1,
                           tol=1e-10)
    x0 = P.cellvec()
    r0 = P.pcg_solve(b, x0, opts)
    P.set_metric_mode(1)
    x1 = P.cellvec()
    r1 = P.pcg_solve(b, x1, opts)
    assert r0["converged"] and r1["converged"] and abs(r0["iters"] - r1["iters"]) <= 1
    assert relerr(host(x1), host(x0)) < 1e-8
    with pytest.raises(fe.FeError):
        fe.Problem(3, 3, 4, bc=1).set_metric_mode(1)


@pytest.mark.parametrize("k,n", [(2, 3), (3, 2)])
def test_general_load_vector(gpu_lib, k, n):
    fe = gpu_lib
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, AMP, coefficient_modes(2))
    P = problem(fe, k, n)
    b = P.cellvec()
    P.rhs_manufactured(b)
    assert relerr(host(b), g.load_vector().ravel()) < 1e-12


@pytest.mark.parametrize("k,n", [(2, 3), (3, 4), (1, 4), (7, 3)])
def test_averaged_patch_inverse(gpu_lib, k, n):
    """Per-patch separable factors (averaged geometry): k <= 3 on the slot-split
    patch kernel, k = 7 on the one-lane-per-pencil kernel with its factors in LDS."""
    fe = gpu_lib
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, AMP, coefficient_modes(2))
    P = problem(fe, k, n)
    r = uniform(m.n_cellwise, seed=301)
    expect = sep_patch_inverse_cellwise(m, averaged_weights(g), r.reshape(m.n_cells, -1)).ravel()
    for dtype, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5)):
        z = P.cellvec(dtype)
        P.patch_inverse(dev(r, dtype), z, factors=1)
        assert relerr(host(z), expect) < tol, (dtype, relerr(host(z), expect))


@pytest.mark.parametrize("smoother,inner,flexible", [(0, 0, 0), (1, 1, 1)])
def test_deformed_pcg_matches_sparse_solve(gpu_lib, smoother, inner, flexible):
    fe = gpu_lib
    k, n = 3, 4
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, AMP, coefficient_modes(2))
    A = assemble_csr(m, g.element_matrices())
    I = np.flatnonzero(~m.boundary_mask_global())
    P = problem(fe, k, n)
    b = P.cellvec()
    P.rhs_manufactured(b)
    x = P.cellvec()
    opts = fe.default_opts(smoother=smoother, inner=inner, flexible=flexible, omega=0.6, factors=1,
                           nu_pre=2 if smoother == 0 else 1, nu_post=2 if smoother == 0 else 1, tol=1e-10)
    rep = P.pcg_solve(b, x, opts)
    assert rep["converged"], rep
    bg = m.assemble(host(b))
    xe = np.zeros(m.n_global)
    xe[I] = spla.spsolve(A[I][:, I].tocsc(), bg[I])
    assert relerr(host(x), m.gather(xe).ravel()) < 1e-7


def test_folding_deformation_is_rejected(gpu_lib):
    fe = gpu_lib
    with pytest.raises(fe.FeError):
        problem_amp = fe.Problem(3, 2, 4, geometry=fe.GEOM_DEFORMED, deform_amp=0.15)
        del problem_amp
    fe.Problem(3, 2, 4, geometry=fe.GEOM_DEFORMED, deform_amp=0.137).close()
