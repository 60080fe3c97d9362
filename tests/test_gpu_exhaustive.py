"""Exhaustive, element-wise GPU parity at the benchmark sizes, in the launch
configurations the benchmark times: every entry of the Q3 64^3 apply and patch
inverse (FP64, FP32) and every cell of the Q7 32^3 apply, against the oracle.

The oracle's plain definitions scale to these sizes when written as dense
batched products: the cell-wise apply is one dense A_K (x_K) per cell; on the
uniform Cartesian mesh every interior vertex patch has the same matrix A_p
(translation invariance: the patch of the single interior vertex of a 2^3
mesh with the same cell size), so the patch inverse is G sum_p R_p^T A_p^{-1}
R_p G^T r with one dense A_p^{-1} applied to all patches at once.

Bounds: norm-wise relative 1e-12 (FP64) / 1e-5 (FP32), and entry-wise
max |got - exp| <= c max |exp| with c = 1e-11 (FP64) / 1e-4 (FP32), so that no
single entry can hide under the norm.
"""
import numpy as np
import pytest
import torch

from oracle.mesh import StructuredMesh
from oracle.operators import boundary_mask_cellwise, element_matrix_cartesian
from oracle.patch import patch_inverse_cartesian
from synthetic_inputs import uniform

pytestmark = pytest.mark.gpu
BOUNDS = {torch.float64: (1e-12, 1e-11), torch.float32: (1e-5, 1e-4)}


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def check(got, expect, dtype, what):
    norm_tol, entry_tol = BOUNDS[dtype]
    rel = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    ent = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
    print("%s %s: norm-wise %.2e, entry-wise %.2e" % (what, dtype, rel, ent), flush=True)
    assert rel < norm_tol, (what, dtype, rel)
    assert ent < entry_tol, (what, dtype, ent)


@pytest.mark.parametrize("k,n", [(3, 64), (7, 32)])
def test_apply_every_entry(gpu_lib, k, n):
    fe = gpu_lib
    print("exhaustive apply", k, n, flush=True)
    m = StructuredMesh(3, k, n)
    x = m.gather(uniform(m.n_global, seed=201))
    mask = boundary_mask_cellwise(m).reshape(m.n_cells, -1)
    A = element_matrix_cartesian(3, k, m.h)
    expect = np.where(mask, 0.0, np.where(mask, 0.0, x) @ A.T)
    P = fe.Problem(3, k, n, bc=1)
    for dtype in (torch.float64, torch.float32):
        y = P.cellvec(dtype)
        P.apply(dev(x, dtype), y)
        check(host(y).reshape(m.n_cells, -1), expect, dtype, "apply Q%d %d^3" % (k, n))
        del y
    P.close()


def test_patch_inverse_every_entry_q3_64(gpu_lib):
    fe = gpu_lib
    k, n = 3, 64
    print("exhaustive patch inverse", k, n, flush=True)
    m = StructuredMesh(3, k, n)
    r = uniform(m.n_cellwise, seed=203)
    expect = patch_inverse_cartesian(m, r.reshape(m.n_cells, -1))
    P = fe.Problem(3, k, n, bc=1)
    for dtype in (torch.float64, torch.float32):
        z = P.cellvec(dtype)
        P.patch_inverse(dev(r, dtype), z)
        check(host(z).reshape(m.n_cells, -1), expect, dtype, "patch inverse Q3 64^3")
        del z
    P.close()
