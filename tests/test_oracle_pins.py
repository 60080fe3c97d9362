"""Pins of oracle parts that the first pins left loose: the deformed load vector
and operator (volume, exact integrals, a manufactured solution on the mapped
domain), the Chebyshev semi-iteration (closed-form error polynomial), Adam
beyond its first step (closed forms of the bias-corrected moments), and the
patch features on an affinely mapped mesh (constant, known Jacobian)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.geometry import DeformedGeometry
from oracle.learned import adam_step, patch_features
from oracle.mesh import StructuredMesh
from oracle.multigrid import chebyshev_sweep
from oracle.operators import assemble_csr
from synthetic_inputs import coefficient_modes, uniform


# ------------------------------------------------------------------ deformed load vector

@pytest.mark.parametrize("k,n", [(2, 2), (2, 3), (3, 2)])
def test_load_vector_of_one_integrates_the_volume(k, n):
    """The isoparametric map fixes the cube's faces (the shift vanishes there), so
    the mapped domain is the unit cube: with f = 1, sum_K sum_i b_K,i = sum_K int_K 1
    = 1 (sum_i phi_i = 1).  det J has degree <= 3k - 1 per direction, which the
    (k+2)-point Gauss rule integrates exactly for k <= 4, so the sum is 1 to rounding.
    A missing det J, a wrong weight or a wrong map fails this."""
    g = DeformedGeometry(StructuredMesh(3, k, n), 0.1, None)
    b = g.load_vector(f=lambda x: np.ones(x.shape[:-1]))
    assert abs(b.sum() - 1.0) < 1e-13
    assert np.all(b.sum(axis=1) > 0)               # every cell has positive volume


def test_load_vector_of_linear_functions_is_exact():
    """int over the unit cube of a + g.x is a + g.(1/2, 1/2, 1/2); at k = 2 the
    integrand x(xi) det J has degree <= 4k - 1 = 7 per direction, exact with 4 points."""
    g = DeformedGeometry(StructuredMesh(3, 2, 3), 0.1, None)
    gv = np.array([0.7, -1.3, 2.1])
    b = g.load_vector(f=lambda x: 0.25 + x @ gv)
    assert abs(b.sum() - (0.25 + 0.5 * gv.sum())) < 1e-13
    # pairing with the nodal interpolant of 1 on one coordinate: sum_i b_K,i x_i(K) = int x_1 f
    # for f = 1 (x_1 is in the Q_k space of the isoparametric map)
    b1 = g.load_vector(f=lambda x: np.ones(x.shape[:-1]))
    assert abs(np.sum(b1 * g.X[..., 0]) - 0.5) < 1e-13


def _deformed_mms_error(k, n, amp):
    m = StructuredMesh(3, k, n)
    g = DeformedGeometry(m, amp, None)
    A = assemble_csr(m, g.element_matrices())
    b = m.assemble(g.load_vector())
    I = np.flatnonzero(~m.boundary_mask_global())
    u = np.zeros(m.n_global)
    u[I] = spla.spsolve(sp.csc_matrix(A[I][:, I]), b[I])
    exact = lambda x: np.prod(np.sin(np.pi * x), axis=-1)
    return g.l2_error(m.gather(u), exact)


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_deformed_manufactured_solution_converges_at_order_k_plus_1(k):
    """-Laplace u = f on the mapped cube (kappa = 1) with u = prod sin(pi x_a), which
    vanishes on the boundary; f = 3 pi^2 u at the physical points.  The Galerkin
    solution's L2 error on the mapped domain falls like h^(k+1) (standard FE
    theory for isoparametric Q_k).  Pins the load vector, the metric and the
    element matrices together: a wrong det J, a transposed J^-1 or a missing
    factor gives O(1) errors or the wrong rate."""
    ns = (2, 4, 8) if k == 2 else (4, 8, 16)
    errs = [_deformed_mms_error(k, n, 0.1) for n in ns]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > k + 1 - 0.35, (errs, rates)
    assert errs[-1] < (2e-3 if k == 2 else 2e-2), errs


# ------------------------------------------------------------------ Chebyshev

class _Diag:
    def __init__(self, lam):
        self.A = sp.diags(lam)


@pytest.mark.parametrize("degree", [1, 2, 3, 4, 5])
def test_chebyshev_sweep_has_the_closed_form_error_polynomial(degree):
    """From u = 0 with the identity preconditioner, the semi-iteration of degree d
    on [a, b] leaves the error e_d = p_d(A) e_0 with
    p_d(lam) = T_d((theta - lam)/delta) / T_d(theta/delta), theta = (a+b)/2,
    delta = (b-a)/2 (Chebyshev polynomial of the first kind).  On a diagonal
    matrix that is a per-eigenvalue scalar identity."""
    lmax, ratio = 3.7, 20.0
    lam = np.concatenate([np.linspace(0.01, lmax, 40), [lmax / ratio, lmax, 0.5 * lmax]])
    b = uniform(len(lam), seed=90 + degree)
    u = chebyshev_sweep(_Diag(lam), b, np.zeros_like(b), lmax, degree, ratio, precond=lambda r: r,
                        u_is_zero=True)
    a = lmax / ratio
    theta, delta = 0.5 * (lmax + a), 0.5 * (lmax - a)

    def T(d, x):   # Chebyshev T_d on any real x (cosh branch outside [-1, 1])
        x = np.asarray(x, dtype=np.float64)
        out = np.empty_like(x)
        inside = np.abs(x) <= 1
        out[inside] = np.cos(d * np.arccos(x[inside]))
        xo = x[~inside]
        out[~inside] = np.sign(xo) ** d * np.cosh(d * np.arccosh(np.abs(xo)))
        return out

    p = T(degree, (theta - lam) / delta) / T(degree, np.array([theta / delta]))[0]
    expect = (1.0 - p) * b / lam
    assert np.max(np.abs(u - expect)) < 1e-13 * np.max(np.abs(expect))
    # inside the interval the error factor is bounded by 1 / T_d(theta / delta)
    sel = (lam >= a - 1e-15)
    bound = 1.0 / T(degree, np.array([theta / delta]))[0]
    assert np.all(np.abs(p[sel]) <= bound * (1 + 1e-12))


# ------------------------------------------------------------------ Adam

B1, B2, EPS = 0.9, 0.999, 1e-8


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient g the bias-corrected moments equal g and g^2 at
    every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so every step moves by
    lr g / (|g| + eps): after t steps p_t = p_0 - t lr g / (|g| + eps).  A missing
    or mis-indexed bias correction breaks it from t = 2 on."""
    p0 = uniform(16, seed=40)
    g = uniform(16, seed=41) + np.sign(uniform(16, seed=41)) * 0.1
    p, m, v = p0.copy(), np.zeros(16), np.zeros(16)
    for t in (1, 2, 3, 4):
        p, m, v = adam_step(p, g, m, v, t, lr=1e-2)
        assert np.allclose(p, p0 - t * 1e-2 * g / (np.abs(g) + EPS), rtol=0, atol=1e-15)


def test_adam_alternating_gradient_steps_two_and_three():
    """Gradients g, -g, g: v_t = (1 - b2^t) g^2 (so v_hat = g^2), m_2 = -(1 - b1)^2 g,
    m_3 = (1 - b1)(1 - b1 + b1^2) g.  Hence step 2 moves by +lr (1 - b1)/(1 + b1)
    sign(g) and step 3 by -lr (1 - b1 + b1^2)/(1 + b1 + b1^2) sign(g):
    +lr/19 and -lr 0.91/2.71 at b1 = 0.9 (eps negligible at |g| >= 0.1)."""
    g = np.array([0.5, -2.0, 0.1, 3.0])
    lr = 1e-2
    p0 = np.zeros(4)
    p1, m, v = adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr=lr)
    p2, m, v = adam_step(p1, -g, m, v, 2, lr=lr)
    assert np.allclose(p2 - p1, lr * (1 / 19) * np.sign(g), rtol=1e-7, atol=0)
    p3, m, v = adam_step(p2, g, m, v, 3, lr=lr)
    assert np.allclose(p3 - p2, -lr * (0.91 / 2.71) * np.sign(g), rtol=1e-7, atol=0)
    # the moments themselves, in closed form
    assert np.allclose(m, (1 - B1) * (1 - B1 + B1 ** 2) * g, rtol=1e-13)
    assert np.allclose(v, (1 - B2 ** 3) * g ** 2, rtol=1e-13)


def test_adam_is_invariant_to_gradient_scale():
    p0 = uniform(8, seed=42)
    gs = [uniform(8, seed=43 + t) for t in range(3)]
    pa, ma, va = p0.copy(), np.zeros(8), np.zeros(8)
    pb, mb, vb = p0.copy(), np.zeros(8), np.zeros(8)
    for t, g in enumerate(gs, start=1):
        pa, ma, va = adam_step(pa, g, ma, va, t, lr=1e-3, eps=0.0)
        pb, mb, vb = adam_step(pb, 1000.0 * g, mb, vb, t, lr=1e-3, eps=0.0)
        assert np.allclose(pa, pb, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ features on an affine mesh

class _AffineGeometry:
    """The structured mesh mapped by x = F xh + c (constant Jacobian F / n per cell);
    only what patch_features reads."""

    def __init__(self, mesh, F, c):
        from oracle.basis import gll_nodes
        xi = gll_nodes(mesh.k)
        ref = (mesh.cell_coords()[:, None, :] + xi[mesh.local_coords()][None]) / mesh.n
        self.mesh = mesh
        self.X = ref @ F.T + c
        self.scale = 1.0


@pytest.mark.parametrize("k,n", [(2, 3), (3, 4)])
def test_features_on_an_affine_mesh(k, n):
    """For x = F xh + c the cell Jacobian is F / n, so n kappa det J J^-1 J^-T =
    det F F^-1 F^-T for every cell (any n), log kappa = 0 and log(n^3 det J) =
    log det F.  F has nonzero off-diagonal entries, so the xy, xz, yz features
    are pinned too (the undeformed mesh leaves them 0)."""
    F = np.array([[1.2, 0.3, -0.1], [0.2, 0.9, 0.25], [-0.15, 0.1, 1.1]])
    g = _AffineGeometry(StructuredMesh(3, k, n), F, np.array([0.1, -0.2, 0.3]))
    f = patch_features(g).reshape(-1, 8, 8)
    Fi = np.linalg.inv(F)
    C = np.linalg.det(F) * Fi @ Fi.T
    expect = np.array([C[0, 0], C[1, 1], C[2, 2], C[0, 1], C[0, 2], C[1, 2], 0.0, np.log(np.linalg.det(F))])
    assert f.shape[0] == (n - 1) ** 3
    assert np.max(np.abs(f - expect[None, None, :])) < 1e-13
    assert min(abs(C[0, 1]), abs(C[0, 2]), abs(C[1, 2])) > 1e-2


def test_cached_coefficient_scale_is_the_oracles():
    """The cached whole-mesh coefficient scales are what the oracle computes (the
    Q3 48^3 entry is recomputed here; both come from the same committed script)."""
    import json
    import os
    from oracle.geometry import coefficient_scale
    from oracle.mesh import StructuredMesh
    from synthetic_inputs import coefficient_modes
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "coef_scale.json")
    with open(path) as f:
        scales = json.load(f)["scales"]
    assert set(scales) == {"3_48_0.1_2", "7_64_0.1_2"}
    s = coefficient_scale(StructuredMesh(3, 3, 48), 0.1, coefficient_modes(2), chunk=512)
    assert s == scales["3_48_0.1_2"]
    # |g| <= sum |a_j|, so s >= 1 / sum |a_j|; the finer mesh samples the same field
    assert all(v >= 1.0 / np.sum(np.abs(coefficient_modes(2)[1])) for v in scales.values())
    assert abs(scales["7_64_0.1_2"] - s) < 1e-3 * s
