"""GPU parity of transfers, smoothers, V-cycle and PCG against the assembled oracle.

The cell-wise V-cycle equals G times the classical assembled V-cycle (paper,
Sec. 3, theorem on the equivalence with local multigrid); transfers satisfy
P_cell G = G P_CG and G^T R_cell = R_CG G^T (Sec. 3.1 lemmas).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle.kron import KroneckerOperator
from oracle.mesh import StructuredMesh
from oracle.multigrid import (Hierarchy, global_prolongation_1d, jacobi_sweep, make_chebyshev_smoother,
                              make_jacobi_smoother, vcycle)
from synthetic_inputs import uniform

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def full_prolongation(k, n_coarse):
    P1 = sp.csr_matrix(global_prolongation_1d(k, n_coarse))
    return sp.kron(P1, sp.kron(P1, P1), format="csr")


def to_cell(level, u_int):
    return level.mesh.gather(level.to_full(u_int)).ravel()


def to_int(level, r_cell):
    return level.to_int(level.mesh.assemble(r_cell))


@pytest.mark.parametrize("k,n", [(1, 4), (2, 4), (3, 4), (7, 2), (4, 8)])
def test_transfers_commute_with_gather(gpu_lib, k, n):
    fe = gpu_lib
    P = fe.Problem(3, k, n, bc=1)
    L = P.n_levels - 1
    mf, mc = StructuredMesh(3, k, n), StructuredMesh(3, k, n // 2)
    Pf = full_prolongation(k, n // 2)
    xcg = uniform(mc.n_global, seed=200)
    ec = dev(mc.gather(xcg).ravel())
    ef = torch.zeros(mf.n_cellwise, dtype=torch.float64, device="cuda")
    P.prolongate_add(L, ec, ef)
    assert relerr(host(ef), mf.gather(Pf @ xcg).ravel()) < 1e-14
    r = uniform(mf.n_cellwise, seed=201)
    v = uniform(mf.n_cellwise, seed=202)
    bc = torch.zeros(mc.n_cellwise, dtype=torch.float64, device="cuda")
    P.restrict_residual(L, dev(r), None, bc)
    assert relerr(mc.assemble(host(bc)), Pf.T @ mf.assemble(r)) < 1e-13
    P.restrict_residual(L, dev(r), dev(v), bc)
    assert relerr(mc.assemble(host(bc)), Pf.T @ mf.assemble(r - v)) < 1e-13


@pytest.mark.parametrize("k,n", [(2, 4), (3, 3)])
def test_jacobi_sweep_equals_classical(gpu_lib, k, n):
    """Lemma verifying the smoother assumption: one fused sweep = G (classical damped Jacobi)."""
    fe = gpu_lib
    h = Hierarchy(3, k, n, n_coarse=n)
    lev = h.levels[-1]
    P = fe.Problem(3, k, n, bc=1, n_coarse=n)
    u0 = uniform(lev.n_int, seed=203)
    b = uniform(lev.mesh.n_cellwise, seed=204)
    u = dev(to_cell(lev, u0))
    v = P.cellvec()
    P.jacobi_sweep(-1, dev(b), u, v, 0.7)
    expect = jacobi_sweep(lev, to_int(lev, b), u0, 0.7)
    assert relerr(host(u), to_cell(lev, expect)) < 1e-13


@pytest.mark.parametrize("k,n", [(2, 4), (3, 4), (2, 8), (7, 2)])
@pytest.mark.parametrize("inner", [0, 1])
def test_jacobi_vcycle_equals_classical(gpu_lib, k, n, inner):
    fe = gpu_lib
    h = Hierarchy(3, k, n)
    P = fe.Problem(3, k, n, bc=1)
    lev = h.levels[-1]
    b = uniform(lev.mesh.n_cellwise, seed=205)
    expect = to_cell(lev, vcycle(h, to_int(lev, b), make_jacobi_smoother(0.7, 2, 2)))
    dtype = torch.float64 if inner == 0 else torch.float32
    opts = fe.default_opts(inner=inner, omega=0.7, nu_pre=2, nu_post=2)
    e = P.cellvec(dtype)
    P.vcycle(dev(b, dtype), e, opts)
    tol = 1e-11 if inner == 0 else 2e-5
    assert relerr(host(e), expect) < tol


@pytest.mark.parametrize("k,n", [(2, 4), (3, 4), (7, 2), (1, 4), (5, 2), (6, 2)])
@pytest.mark.parametrize("inner", [0, 1])
def test_chebyshev_fdm_vcycle_equals_classical(gpu_lib, k, n, inner):
    """Covers every summing pass that carries the Chebyshev step: k = 1 (slot
    layout), k = 5, 6, 7 (patch-major), and k = 2, 3 with the fused inverse plus a
    separate update."""
    fe = gpu_lib
    h = Hierarchy(3, k, n)
    P = fe.Problem(3, k, n, bc=1)
    lev = h.levels[-1]
    lhat = 2.04   # top of the Chebyshev interval handed to both sides; interval [lhat / 20, lhat]
    b = uniform(lev.mesh.n_cellwise, seed=206)
    sm = make_chebyshev_smoother([lhat] * len(h.levels), degree=3, ratio=20.0, nu_pre=1, nu_post=1)
    expect = to_cell(lev, vcycle(h, to_int(lev, b), sm))
    dtype = torch.float64 if inner == 0 else torch.float32
    opts = fe.default_opts(inner=inner, smoother=fe.SMOOTH_CHEB_FDM, cheb_degree=3, cheb_ratio=20.0,
                           cheb_lmax=lhat, nu_pre=1, nu_post=1)
    e = P.cellvec(dtype)
    P.vcycle(dev(b, dtype), e, opts)
    tol = 1e-11 if inner == 0 else 2e-5
    assert relerr(host(e), expect) < tol


def test_lmax_estimate_brackets_exact(gpu_lib):
    fe = gpu_lib
    k, n = 3, 4
    h = Hierarchy(3, k, n)
    lev = h.levels[-1]
    A = lev.A.toarray()
    PA = np.stack([lev.patch_inverse(A[:, j], shared=True) for j in range(A.shape[1])], axis=1)
    exact = np.max(np.real(np.linalg.eigvals(PA)))
    P = fe.Problem(3, k, n, bc=1)
    est = P.estimate_lmax(-1, steps=15)
    assert 0.9 * exact < est <= exact * (1 + 1e-8), (est, exact)


def test_jacobi_lmax_estimate_and_auto_damping(gpu_lib):
    """lambda_max(D^-1 A) by Lanczos brackets the dense value; omega = 0 selects
    4 / (3 lambda_max) per level and the resulting PCG converges."""
    fe = gpu_lib
    k, n = 3, 4
    h = Hierarchy(3, k, n)
    A = h.levels[-1].A.toarray()
    exact = np.max(np.linalg.eigvalsh(A / np.sqrt(np.outer(np.diag(A), np.diag(A)))))
    P = fe.Problem(3, k, n, bc=1)
    est = P.estimate_lmax(-1, steps=15, smoother=fe.SMOOTH_JACOBI)
    assert 0.9 * exact < est <= exact * (1 + 1e-8), (est, exact)
    P8 = fe.Problem(3, k, 8, bc=1)
    b = P8.cellvec()
    P8.rhs_manufactured(b)
    x = P8.cellvec()
    rep = P8.pcg_solve(b, x, fe.default_opts(omega=0.0))
    assert rep["converged"] and rep["iters"] <= 30


@pytest.mark.parametrize("smoother,inner,flexible", [(0, 0, 0), (1, 0, 0), (1, 1, 1), (0, 1, 1)])
def test_pcg_reaches_exact_discrete_solution(gpu_lib, smoother, inner, flexible):
    fe = gpu_lib
    k, n = 3, 8
    m = StructuredMesh(3, k, n)
    ko = KroneckerOperator(3, k, n)
    P = fe.Problem(3, k, n, bc=1)
    b = P.cellvec()
    P.rhs_manufactured(b)
    x = P.cellvec()
    opts = fe.default_opts(smoother=smoother, inner=inner, flexible=flexible, tol=1e-10,
                           nu_pre=2 if smoother == 0 else 1, nu_post=2 if smoother == 0 else 1)
    rep = P.pcg_solve(b, x, opts)
    assert rep["converged"] and rep["relres"] <= 1e-10
    assert rep["iters"] <= 30
    bmask = m.boundary_mask_global()
    bg = m.assemble(host(b))
    xe = np.zeros(m.n_global)
    xe[~bmask] = ko.solve(bg[~bmask])
    xs = host(x)
    assert relerr(xs, m.gather(xe).ravel()) < 1e-7


def test_rhs_matches_oracle(gpu_lib):
    from oracle.rhs import load_vector_cartesian
    fe = gpu_lib
    for dim, k, n in [(3, 3, 4), (3, 7, 2), (2, 2, 16)]:
        m = StructuredMesh(dim, k, n)
        P = fe.Problem(dim, k, n, bc=1)
        b = P.cellvec()
        P.rhs_manufactured(b)
        assert relerr(host(b), load_vector_cartesian(m).ravel()) < 1e-13


def test_pcg_error_paths(gpu_lib):
    fe = gpu_lib
    P = fe.Problem(3, 2, 4, bc=1)
    b = P.cellvec()
    P.rhs_manufactured(b)
    x = P.cellvec()
    rep = P.pcg_solve(b, x, fe.default_opts(maxit=1), raise_on_error=False)
    assert rep["status"] == "FE_ENOTCONV" and rep["iters"] == 1
    x.zero_()
    rep = P.pcg_solve(b, x, fe.default_opts(omega=-0.7), raise_on_error=False)
    assert rep["status"] == "FE_EBREAKDOWN"
    bad = b.clone()
    bad[13] = float("nan")   # local node (1,1,1) of cell 0: an interior node for k = 2
    x.zero_()
    rep = P.pcg_solve(bad, x, fe.default_opts(), raise_on_error=False)
    assert rep["status"] == "FE_EBREAKDOWN"
    with pytest.raises(fe.FeError):
        P.pcg_solve(b, x, fe.default_opts(smoother=5))


@pytest.mark.parametrize("smoother,inner,flexible,k,n", [(1, 1, 1, 3, 8), (0, 0, 0, 3, 8), (1, 1, 1, 7, 4)])
def test_pcg_graph_replay_matches_eager(gpu_lib, smoother, inner, flexible, k, n):
    """The preconditioner replayed as a HIP graph gives the eager solve bit for bit:
    same iteration count and identical solution, over several solves in a row (each
    replaying the graph many times, with the solver's own synchronizations between
    replays), also after an option change that must drop the captured graph."""
    fe = gpu_lib
    P = fe.Problem(3, k, n, bc=1)
    b = P.cellvec()
    P.rhs_manufactured(b)
    nu = 2 if smoother == 0 else 1
    opts = fe.default_opts(smoother=smoother, inner=inner, flexible=flexible, tol=1e-10, nu_pre=nu, nu_post=nu)
    opts2 = fe.default_opts(smoother=smoother, inner=inner, flexible=flexible, tol=1e-10, nu_pre=2 * nu,
                            nu_post=2 * nu)

    def solve(o):
        x = P.cellvec()
        rep = P.pcg_solve(b, x, o)
        assert rep["converged"], rep
        return rep["iters"], host(x)

    try:
        fe.set_graphs(False)
        it_e, x_e = solve(opts)
        it2_e, x2_e = solve(opts2)
        fe.set_graphs(True)
        for o, it_ref, x_ref in ((opts, it_e, x_e), (opts, it_e, x_e), (opts2, it2_e, x2_e), (opts, it_e, x_e)):
            it_g, x_g = solve(o)
            assert it_g == it_ref
            assert np.array_equal(x_g, x_ref)
        # a V-cycle with an odd number of sweeps between two replayed solves (with
        # Jacobi the levels' iterate and scratch buffers trade places): the next
        # solve must not replay a graph captured on the old buffers
        dt = torch.float64 if inner == 0 else torch.float32
        e1 = P.cellvec(dt)
        P.vcycle(b.to(dt), e1, fe.default_opts(smoother=smoother, inner=inner, flexible=flexible, nu_pre=1,
                                               nu_post=2))
        it_g, x_g = solve(opts)
        assert it_g == it_e
        assert np.array_equal(x_g, x_e)
    finally:
        fe.set_graphs(True)
