"""GPU parity at the benchmark sizes, in the launch configurations the benchmark times.

The oracle cannot form these operators whole, so it checks outputs one by one:

* cell-wise apply on sampled cells (dense A_K x_K, boundary copies masked);
* patch inverse on every node of sampled cells: the sum, over the vertex
  patches that contain the node, of the dense A_p^{-1} R_p G^T r (on a uniform
  Cartesian mesh every interior patch matrix is the one of a 2 x 2 x 2-cell
  mesh with the same cell size);
* general (deformed, variable coefficient) apply on sampled cells, the
  coefficient scale taken over every Gauss point of the whole mesh;
* the MG-PCG solution against the exact discrete solution of the Kronecker
  oracle.

Inputs are seeded synthetic vectors (synthetic_inputs); nothing expected comes
from the GPU path.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from oracle.geometry import DeformedGeometry, coefficient_scale
from oracle.kron import KroneckerOperator
from oracle.mesh import StructuredMesh
from oracle.operators import assemble_csr, boundary_mask_cellwise, element_matrix_cartesian
from oracle.patch import patch_matrices
from oracle.rhs import load_vector_cartesian
from synthetic_inputs import coefficient_modes, rng, uniform

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


ENTRY_TOL = {torch.float64: 1e-11, torch.float32: 1e-4}


def assert_close(got, expect, dtype, tol):
    """Norm-wise relative error below tol and max |got - exp| <= c max |exp|."""
    rel = relerr(got, expect)
    ent = np.max(np.abs(got - expect)) / max(np.max(np.abs(expect)), 1e-300)
    assert rel < tol, (dtype, rel)
    assert ent < ENTRY_TOL[dtype], (dtype, ent)


def sample_cells(n, count, seed):
    """The 8 corner cells, cells on each face and edge, and random cells."""
    c = [0, n - 1]
    picks = {(x, y, z) for x in c for y in c for z in c}
    g = rng(seed)
    while len(picks) < count // 2:
        p = list(g.integers(0, n, size=3))
        p[int(g.integers(0, 3))] = int(g.choice(c))
        picks.add(tuple(int(v) for v in p))
    while len(picks) < count:
        picks.add(tuple(int(v) for v in g.integers(0, n, size=3)))
    return np.array(sorted(x + n * (y + n * z) for x, y, z in picks), dtype=np.int64)


def boundary_mask_at_cells(k, n, cells):
    """True for the copies, in the listed cells, of nodes on the boundary of the cube."""
    K = k + 1
    i = np.arange(K ** 3)
    loc = np.stack([i % K, (i // K) % K, i // (K * K)], axis=1)
    cc = np.stack([cells % n, (cells // n) % n, cells // (n * n)], axis=1)
    g = k * cc[:, None, :] + loc[None, :, :]
    return np.any((g == 0) | (g == k * n), axis=2)


def patch_inverse_at_cells(k, n, r_glob, cells):
    """Oracle patch inverse on the nodes of the listed cells: (len(cells), K^3)."""
    K, M = k + 1, 2 * k - 1
    N = k * n + 1
    small = StructuredMesh(3, k, 2)
    Ap = patch_matrices(assemble_csr(small, element_matrix_cartesian(3, k, 1.0 / n)), small)[0]
    Ainv = sla.inv(Ap)
    off = np.arange(1, M + 1)
    cache = {}

    def patch_solution(v):
        if v not in cache:
            vx, vy, vz = v
            gx, gy, gz = k * (vx - 1) + off, k * (vy - 1) + off, k * (vz - 1) + off
            idx = (gx[None, None, :] + N * (gy[None, :, None] + N * gz[:, None, None])).ravel()
            cache[v] = (Ainv @ r_glob[idx]).reshape(M, M, M)
        return cache[v]

    def containing(g):
        # vertices v with k(v-1) < g < k(v+1), 1 <= v <= n-1, and the patch-local offset
        out = []
        for v in (g // k, g // k + 1):
            if 1 <= v <= n - 1 and k * (v - 1) < g < k * (v + 1):
                out.append((v, g - k * (v - 1) - 1))
        return out

    res = np.zeros((len(cells), K ** 3))
    for ci, e in enumerate(cells):
        cx, cy, cz = e % n, (e // n) % n, e // (n * n)
        for iz in range(K):
            for iy in range(K):
                for ix in range(K):
                    s = 0.0
                    for vz, oz in containing(k * cz + iz):
                        for vy, oy in containing(k * cy + iy):
                            for vx, ox in containing(k * cx + ix):
                                s += patch_solution((vx, vy, vz))[oz, oy, ox]
                    res[ci, ix + K * (iy + K * iz)] = s
    return res


@pytest.mark.parametrize("k,n", [(3, 64), (7, 32)])
def test_apply_full_size(gpu_lib, k, n):
    fe = gpu_lib
    m = StructuredMesh(3, k, n)
    x = m.gather(uniform(m.n_global, seed=201))
    cells = sample_cells(n, 64, seed=202)
    A = element_matrix_cartesian(3, k, m.h)
    mask = boundary_mask_at_cells(k, n, cells)
    assert np.array_equal(mask, boundary_mask_cellwise(m).reshape(m.n_cells, -1)[cells])
    xs = np.where(mask, 0.0, x[cells])
    expect = np.where(mask, 0.0, xs @ A.T)
    P = fe.Problem(3, k, n, bc=1)
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        y = P.cellvec(dtype)
        P.apply(dev(x, dtype), y)
        got = host(y).reshape(m.n_cells, -1)[cells]
        assert_close(got, expect, dtype, tol)
    P.close()


@pytest.mark.parametrize("k,n", [(3, 64), (3, 96), (7, 32)])
def test_patch_inverse_full_size(gpu_lib, k, n):
    """Sampled cells at the benchmark sizes, and Q3 at 96^3 (several z chunks of
    the lattice kernel per column of tiles, 16 x 11 tiles of 7 x 10 patches)."""
    fe = gpu_lib
    m = StructuredMesh(3, k, n)
    r = uniform(m.n_cellwise, seed=203)
    cells = sample_cells(n, 32 if k == 3 else 16, seed=204)
    expect = patch_inverse_at_cells(k, n, m.assemble(r), cells)
    P = fe.Problem(3, k, n, bc=1)
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        z = P.cellvec(dtype)
        P.patch_inverse(dev(r, dtype), z)
        got = host(z).reshape(m.n_cells, -1)[cells]
        assert_close(got, expect, dtype, tol)
    P.close()


@pytest.mark.parametrize("n", [2, 8, 9, 11, 16, 17, 30, 31, 33, 34, 40])
def test_patch_inverse_tile_seams(gpu_lib, n):
    """Q3 at sizes that place the x-tile, y-tile and z-chunk seams of the
    blocked kernel differently (one tile; a tile exactly full; one patch more;
    a last tile that mostly overlaps the one before; a partial last tile;
    tiles of 7 patches (6 cells) along x and 10 (9) along y): sampled cells on and
    next to every seam against the oracle, and bit-identical copies everywhere."""
    fe = gpu_lib
    k = 3
    m = StructuredMesh(3, k, n)
    r = uniform(m.n_cellwise, seed=206)
    g = rng(207)
    xs = sorted({c for c in (0, 1, 5, 6, 7, 11, 12, 13, 14, 15, 16, 27, 28, 29, 30, 31, 32, 33, n - 2, n - 1)
                 if 0 <= c < n})
    ys = sorted({c for c in (0, 1, 8, 9, 10, 17, 18, 19, 27, 28, n - 2, n - 1) if 0 <= c < n})
    cells = {x + n * (y + n * int(g.integers(0, n))) for x in xs for y in ys}
    cells |= {x + n * (y + n * z) for x in xs for y in (0, n - 1) for z in (0, n - 1)}
    cells = np.array(sorted(cells), dtype=np.int64)
    expect = patch_inverse_at_cells(k, n, m.assemble(r), cells)
    P = fe.Problem(3, k, n, bc=1)
    idx = m.global_index_map().ravel()
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        z = P.cellvec(dtype)
        P.patch_inverse(dev(r, dtype), z)
        zh = host(z)
        got = zh.reshape(m.n_cells, -1)[cells]
        assert_close(got, expect, dtype, tol)
        first = np.full(m.n_global, np.nan)
        first[idx[::-1]] = zh[::-1]
        assert np.array_equal(zh, first[idx])
    P.close()


def cached_coefficient_scale(k, n, amp, seed):
    """The whole-mesh coefficient scale, written by tests/golden/make_coef_scale.py
    (which calls only the oracle); recomputed by the oracle when not listed."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "coef_scale.json")
    with open(path) as f:
        scales = json.load(f)["scales"]
    key = "%d_%d_%g_%d" % (k, n, amp, seed)
    if key in scales:
        return scales[key]
    return coefficient_scale(StructuredMesh(3, k, n), amp, coefficient_modes(seed))


@pytest.mark.parametrize("k,n", [(3, 48), (7, 64)])
def test_general_apply_full_size(gpu_lib, k, n):
    """The deformed benchmark meshes with the benchmark's coefficient field."""
    fe = gpu_lib
    amp = 0.1
    m = StructuredMesh(3, k, n)
    coef = coefficient_modes(2)
    scale = cached_coefficient_scale(k, n, amp, 2)
    cells = sample_cells(n, 24, seed=205)
    g = DeformedGeometry(m, amp, coef, scale=scale, cells=cells)
    x = uniform(m.n_cellwise, seed=7).reshape(m.n_cells, -1)
    mask = boundary_mask_at_cells(k, n, cells)
    expect = np.where(mask, 0.0, g.apply(np.where(mask, 0.0, x[cells])))
    P = fe.Problem(3, k, n, geometry=fe.GEOM_DEFORMED, bc=1, deform_amp=amp, coef=coef)
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        y = P.cellvec(dtype)
        P.apply(dev(x, dtype), y)
        got = host(y).reshape(m.n_cells, -1)[cells]
        assert_close(got, expect, dtype, tol)
    P.close()


def test_pcg_q7_32_matches_exact_discrete_solution(gpu_lib):
    """FP32 Chebyshev(3) patch-FDM V-cycle inside flexible FP64 CG, as benchmarked."""
    fe = gpu_lib
    k, n = 7, 32
    m = StructuredMesh(3, k, n)
    b = load_vector_cartesian(m)
    bmask = m.boundary_mask_global()
    bg = m.assemble(b)
    xe = np.zeros(m.n_global)
    xe[~bmask] = KroneckerOperator(3, k, n).solve(bg[~bmask])
    P = fe.Problem(3, k, n, bc=1)
    x = P.cellvec()
    opts = fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F32, flexible=1, nu_pre=1, nu_post=1, tol=1e-10)
    rep = P.pcg_solve(dev(b), x, opts)
    assert rep["converged"] and rep["relres"] <= 1e-10
    assert rep["iters"] <= 15
    assert relerr(host(x), m.gather(xe).ravel()) < 1e-7
    P.close()
