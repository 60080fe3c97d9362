"""Pins for the learned-factor oracle: gradient check, separable fit, gauge, features."""
import numpy as np
import pytest

from oracle.geometry import DeformedGeometry
from oracle.learned import (N_PARAMS, adam_step, best_fit, fit_targets, forward, gauge_fix,
                            gauge_null_space, loss_and_grad, patch_features)
from oracle.mesh import StructuredMesh
from oracle.operators import assemble_csr
from oracle.patch import patch_matrices
from oracle.sepfit import averaged_weights, design_matrix, sep_matrix
from synthetic_inputs import coefficient_modes, uniform


def test_param_count_and_gradient_by_central_differences():
    assert N_PARAMS == 64 * 64 + 64 + 64 * 64 + 64 + 12 * 64 + 12
    p = uniform(N_PARAMS, seed=1) * 0.2
    X = uniform(5 * 64, seed=2).reshape(5, 64)
    T = uniform(5 * 12, seed=3).reshape(5, 12)
    _, g = loss_and_grad(p, X, T)
    rng = np.random.default_rng(0)
    for i in rng.choice(N_PARAMS, 40, replace=False):
        e = np.zeros(N_PARAMS)
        e[i] = 1e-6
        fd = (loss_and_grad(p + e, X, T)[0] - loss_and_grad(p - e, X, T)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10


def test_adam_first_step_moves_by_lr_times_sign():
    p = uniform(10, seed=4)
    g = uniform(10, seed=5)
    q, m, v = adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=1e-3)
    assert np.allclose(q, p - 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-15)


def test_gauge_directions_leave_the_separable_operator_unchanged():
    N = gauge_null_space()
    assert np.allclose(design_matrix() @ N, 0)
    w = np.exp(uniform(12, seed=6) * 0.3)
    t = np.log(w)
    for d in range(3):
        w2 = np.exp(t + 0.37 * N[:, d])
        assert np.allclose(sep_matrix(2, w), sep_matrix(2, w2), rtol=1e-12, atol=1e-14)
    assert np.allclose(gauge_fix(t) @ N, 0, atol=1e-14)


def test_best_fit_recovers_an_exactly_separable_patch():
    k = 2
    w_true = np.exp(uniform(12, seed=7) * 0.4)
    A = sep_matrix(k, w_true)
    w = best_fit(A, k, np.ones(12), sweeps=60)
    assert np.linalg.norm(sep_matrix(k, w) - A) < 1e-8 * np.linalg.norm(A)


def test_best_fit_improves_on_averaged_weights_and_targets_vanish_on_cartesian():
    m = StructuredMesh(3, 2, 3)
    g = DeformedGeometry(m, 0.1, coefficient_modes(3))
    A = assemble_csr(m, g.element_matrices())
    P = patch_matrices(A, m)
    w0 = averaged_weights(g)
    for p in range(P.shape[0]):
        w = best_fit(P[p], 2, w0[p], sweeps=30)
        assert np.linalg.norm(sep_matrix(2, w) - P[p]) <= np.linalg.norm(sep_matrix(2, w0[p]) - P[p]) + 1e-14
    mc = StructuredMesh(3, 2, 3)
    gc = DeformedGeometry(mc, 0.0, None)
    t = fit_targets(gc, assemble_csr(mc, gc.element_matrices()), sweeps=5)
    assert np.max(np.abs(t)) < 1e-10


def test_features_on_cartesian_cells():
    m = StructuredMesh(3, 3, 2)
    g = DeformedGeometry(m, 0.0, None)
    f = patch_features(g).reshape(-1, 8, 8)
    assert np.allclose(f[:, :, :3], 1.0, atol=1e-13) and np.allclose(f[:, :, 3:], 0.0, atol=1e-13)
