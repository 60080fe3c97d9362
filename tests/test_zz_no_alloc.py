"""The allocation-free patch inverse (patch_fdm_inverse_noalloc, called through
the C ABI) against the allocating entry point on the same inputs: the same
kernels, so the outputs must agree bit for bit.  Two calls in a row, the second
on a smaller input, per case; size and set-up errors are rejected before any
launch."""
import ctypes

import numpy as np
import pytest
import torch

from synthetic_inputs import coefficient_modes, uniform

pytestmark = pytest.mark.gpu


def _noalloc(fe, P, level, r, z, factors=0):
    return fe._lib.patch_fdm_inverse_noalloc(P.h, level, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                             fe.F64 if r.dtype == torch.float64 else fe.F32, factors,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _pair(fe, P, level, dtype, seed, factors=0):
    n_len = P.len if level == -1 else P.level_len(level)
    r = torch.as_tensor(uniform(n_len, seed=seed), dtype=dtype, device="cuda")
    z_ref = torch.full((n_len,), float("nan"), dtype=dtype, device="cuda")
    z = torch.full((n_len,), float("nan"), dtype=dtype, device="cuda")
    P.patch_inverse(r, z_ref, factors=factors, level=level)
    st = _noalloc(fe, P, level, r, z, factors)
    torch.cuda.synchronize()
    assert st == 0, fe.last_error()
    assert torch.isfinite(z).all()
    assert torch.equal(z, z_ref)
    return z


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_patch_inverse_q7(gpu_lib, dtype):
    fe = gpu_lib
    print("noalloc Q7 n=8 then n=4", dtype, flush=True)
    P = fe.Problem(3, 7, 8, bc=1)
    _pair(fe, P, -1, dtype, seed=501)          # 343 patches, patch-major scratch
    Q = fe.Problem(3, 7, 4, bc=1)
    _pair(fe, Q, -1, dtype, seed=502)          # smaller input, same array
    _pair(fe, P, 1, dtype, seed=503)           # a coarser level of the first problem


def test_noalloc_2d_and_fused(gpu_lib):
    fe = gpu_lib
    print("noalloc 2D Q2 n=16, 3D Q3 n=8 (one-pass kernel)", flush=True)
    _pair(fe, fe.Problem(2, 2, 16, bc=1), -1, torch.float64, seed=504)
    _pair(fe, fe.Problem(3, 3, 8, bc=1), -1, torch.float64, seed=505)


def test_noalloc_per_patch_factors(gpu_lib):
    fe = gpu_lib
    print("noalloc deformed Q3 n=6 then n=4, averaged factors", flush=True)
    for n, seed in ((6, 506), (4, 507)):
        P = fe.Problem(3, 3, n, geometry=fe.GEOM_DEFORMED, bc=1, deform_amp=0.1, coef=coefficient_modes(3))
        r = torch.as_tensor(uniform(P.len, seed=seed), dtype=torch.float64, device="cuda")
        z = P.cellvec()
        # per-patch factors not set up yet: rejected, nothing launched
        assert _noalloc(fe, P, -1, r, z, factors=1) == -1
        assert "fe_patch_prepare" in fe.last_error()
        P.patch_prepare(torch.float64, factors=1)
        _pair(fe, P, -1, torch.float64, seed=seed, factors=1)


def test_noalloc_rejects_oversize(gpu_lib):
    fe = gpu_lib
    print("noalloc size limit", flush=True)
    assert fe._lib.fe_noalloc_scratch_bytes() == 64 << 20
    P = fe.Problem(3, 7, 16, bc=1)       # 3375 patches x 8 x 343 x 8 B = 74 MB > 64 MiB
    r = torch.ones(P.len, dtype=torch.float64, device="cuda")
    z = torch.zeros(P.len, dtype=torch.float64, device="cuda")
    assert _noalloc(fe, P, -1, r, z) == -1
    assert "exceeds" in fe.last_error()
    assert torch.count_nonzero(z).item() == 0
    # the FP32 scratch of the same mesh (37 MB) fits
    _pair(fe, P, -1, torch.float32, seed=508)
