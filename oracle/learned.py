"""Learned per-patch 1D factors: features, best-fit targets, reference MLP (oracle; test infrastructure).

Readings (the paper has no learned component; these define it for this
workload):

* features of a patch: for each of its 8 cells (slot s = sx + 2 sy + 4 sz)
  the 6 entries (xx, yy, zz, xy, xz, yz) of n * kappa det(J) J^{-1} J^{-T} at
  the cell centre, log kappa at the centre and log(n^3 det J) at the centre:
  64 inputs;
* target of a patch: the 12 log-weights of the best Kronecker-sum fit
  min ||A_p - A_sep(w)||_F (alternating linear least squares from the
  averaged-geometry weights, a fixed number of sweeps), with the three
  scaling gauges removed (projection orthogonal to the null space of the
  log-space design matrix) after subtracting log(h)/3, so that a Cartesian
  patch of any size has target 0;
* network: 64 -> 64 -> 64 -> 12, tanh hidden layers, linear output, loss =
  mean squared error over batch and outputs; Adam (beta1 0.9, beta2 0.999,
  eps 1e-8).
"""
import numpy as np

from .basis import mass_1d, stiffness_1d
from .geometry import coefficient_raw, tensor_basis
from .patch import patch_matrices
from .sepfit import averaged_weights, design_matrix, patch_cells

N_IN, N_HID, N_OUT = 64, 64, 12
SIZES = [(N_HID, N_IN), (N_HID, N_HID), (N_OUT, N_HID)]
N_PARAMS = sum(o * i + o for o, i in SIZES)


# ------------------------------------------------------------------ features

def patch_features(geom, modes=None, amps=None, phases=None):
    """(n_patches, 64) features of every patch of the geometry's mesh."""
    m = geom.mesh
    V, Gr = tensor_basis(m.k, np.array([0.5]))
    xc = np.einsum("qj,ejd->eqd", V, geom.X)[:, 0]                   # (E, 3)
    J = np.einsum("qja,ejd->eqda", Gr, geom.X)[:, 0]                # (E, 3, 3)
    det = np.linalg.det(J)
    if amps is not None and len(amps):
        kap = np.exp(geom.scale * coefficient_raw(xc, np.asarray(modes), np.asarray(amps), np.asarray(phases)))
    else:
        kap = np.ones(len(det))
    Ji = np.linalg.inv(J)
    C = (m.n * kap * det)[:, None, None] * np.einsum("ead,ebd->eab", Ji, Ji)
    cell_f = np.stack([C[:, 0, 0], C[:, 1, 1], C[:, 2, 2], C[:, 0, 1], C[:, 0, 2], C[:, 1, 2],
                       np.log(kap), np.log(det * m.n ** 3)], axis=1)  # (E, 8)
    cells = patch_cells(m)
    return cell_f[cells].reshape(len(cells), 64)


# ------------------------------------------------------------------ best Kronecker-sum fit

def pieces_1d(k):
    """Interior restrictions of [D on interval 0, D on interval 1, B on 0, B on 1]."""
    B, D = mass_1d(k), stiffness_1d(k)
    N = 2 * k + 1
    out = []
    for mat in (D, B):
        for e in range(2):
            P = np.zeros((N, N))
            P[k * e:k * e + k + 1, k * e:k * e + k + 1] = mat
            out.append(P[1:-1, 1:-1])
    return out   # D0, D1, B0, B1


def _factors(E, w):
    K = [w[2 * d] * E[0] + w[2 * d + 1] * E[1] for d in range(3)]
    M = [w[6 + 2 * d] * E[2] + w[7 + 2 * d] * E[3] for d in range(3)]
    return K, M


def _kron3(X, Y, Z):
    """Dense operator acting with X along x, Y along y, Z along z (x fastest)."""
    return np.kron(Z, np.kron(Y, X))


def best_fit(Ap, k, w0, sweeps=30):
    """Alternating least squares for min ||Ap - A_sep(w)||_F, starting from w0."""
    E = pieces_1d(k)
    w = np.array(w0, dtype=np.float64)
    a = Ap.ravel()
    for _ in range(sweeps):
        K, M = _factors(E, w)
        # stiffness weights of all three directions (linear with the masses fixed)
        cols = []
        for d in range(3):
            for c in range(2):
                ops = [M[0], M[1], M[2]]
                ops[d] = E[c]
                cols.append(_kron3(*ops).ravel())
        sol = np.linalg.lstsq(np.stack(cols, 1), a, rcond=None)[0]
        w[:6] = np.maximum(sol, 1e-12 * np.abs(sol).max())
        # mass weights, one direction at a time
        for d in range(3):
            K, M = _factors(E, w)
            ops0 = [M[0], M[1], M[2]]
            ops0[d] = K[d]
            fixed = _kron3(*ops0).ravel()           # the term with the stiffness along d
            cols = []
            for c in range(2):
                t = np.zeros_like(fixed)
                for e in range(3):
                    if e == d:
                        continue
                    ops = [M[0], M[1], M[2]]
                    ops[e] = K[e]
                    ops[d] = E[2 + c]
                    t += _kron3(*ops).ravel()
                cols.append(t)
            sol = np.linalg.lstsq(np.stack(cols, 1), a - fixed, rcond=None)[0]
            w[6 + 2 * d:8 + 2 * d] = np.maximum(sol, 1e-12 * np.abs(sol).max())
    return w


def gauge_null_space():
    """(12, 3) basis of the scaling gauges of the log-weights."""
    N = np.zeros((12, 3))
    for d in range(3):
        N[6 + 2 * d:8 + 2 * d, d] = 1.0
        for e in range(3):
            if e != d:
                N[2 * e:2 * e + 2, d] = -1.0
    return N


def gauge_fix(theta):
    N = gauge_null_space()
    return theta - (theta @ N) @ np.linalg.solve(N.T @ N, N.T)


def fit_targets(geom, A_csr, sweeps=30):
    """(n_patches, 12) normalized log-weights of the best Kronecker-sum fit."""
    m = geom.mesh
    w0 = averaged_weights(geom)
    P = patch_matrices(A_csr, m)
    out = np.empty((P.shape[0], 12))
    for p in range(P.shape[0]):
        w = best_fit(P[p], m.k, w0[p], sweeps)
        out[p] = gauge_fix(np.log(w) - np.log(m.h) / 3.0)
    assert np.linalg.matrix_rank(design_matrix()) == 9
    return out


def weights_from_targets(t, h):
    return np.exp(np.asarray(t) + np.log(h) / 3.0)


# ------------------------------------------------------------------ MLP

def unpack(params):
    out, o = [], 0
    for (no, ni) in SIZES:
        W = params[o:o + no * ni].reshape(no, ni)
        o += no * ni
        b = params[o:o + no]
        o += no
        out.append((W, b))
    return out


def forward(params, X):
    (W1, b1), (W2, b2), (W3, b3) = unpack(np.asarray(params, dtype=np.float64))
    a1 = np.tanh(X @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    return a2 @ W3.T + b3, (a1, a2)


def loss_and_grad(params, X, T):
    """MSE loss and its gradient by manual backpropagation."""
    params = np.asarray(params, dtype=np.float64)
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    Y, (a1, a2) = forward(params, X)
    nb = X.shape[0]
    diff = Y - T
    loss = np.mean(diff ** 2)
    d3 = 2.0 * diff / (nb * N_OUT)
    gW3, gb3 = d3.T @ a2, d3.sum(0)
    d2 = (d3 @ W3) * (1 - a2 ** 2)
    gW2, gb2 = d2.T @ a1, d2.sum(0)
    d1 = (d2 @ W2) * (1 - a1 ** 2)
    gW1, gb1 = d1.T @ X, d1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; t is the 1-based step count.  Returns (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad ** 2
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
