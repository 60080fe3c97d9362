"""1D reference basis on [0, 1] (oracle; test infrastructure only).

The discretization uses continuous tensor-product Q_p elements with a
Gauss-Lobatto nodal basis (paper, Sec. 2, model problem).  Everything here
is in float64 and follows the plain definitions:

* GLL nodes: 0, 1 and the roots of P_k' (Legendre derivative) mapped to
  [0, 1].
* Lagrange basis by the product formula (no Vandermonde matrices).
* B_ij = int_0^1 phi_i phi_j, D_ij = int_0^1 phi_i' phi_j' by Gauss-Legendre
  quadrature with k+1 points, which integrates both exactly (reading of the
  paper: consistent mass, not GLL collocation).
* 1D prolongation matrices (paper, Sec. 3.1, Inter-grid transfer
  operations): child c in {0, 1} of a parent interval occupies
  [c/2, (c+1)/2]; (P_c)_ij = phi_j((xi_i + c) / 2).
"""
import numpy as np


def legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) on [-1, 1] by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if n == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    dp_prev = np.zeros_like(x)
    dp = np.ones_like(x)
    for m in range(1, n):
        p_next = ((2 * m + 1) * x * p - m * p_prev) / (m + 1)
        dp_next = dp_prev + (2 * m + 1) * p
        p_prev, p = p, p_next
        dp_prev, dp = dp, dp_next
    return p, dp


def gll_nodes(k):
    """Gauss-Lobatto-Legendre nodes of degree k on [0, 1], ascending.

    Interior nodes are the roots of P_k'.  They are found by Newton's method
    on q(x) = (1 - x^2) P_k'(x), whose derivative is -k(k+1) P_k(x), starting
    from the Chebyshev-Gauss-Lobatto points.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    x = -np.cos(np.pi * np.arange(k + 1) / k)
    for _ in range(100):
        p, dp = legendre_and_derivative(k, x[1:-1])
        q = (1.0 - x[1:-1] ** 2) * dp
        dq = -k * (k + 1) * p
        step = q / dq
        x[1:-1] -= step
        if np.max(np.abs(step), initial=0.0) < 1e-17:
            break
    x[0], x[-1] = -1.0, 1.0
    return 0.5 * (x + 1.0)


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [0, 1] (points ascending, weights)."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, j] = phi_j(x_q) for the Lagrange basis on ``nodes`` (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_derivatives(nodes, x):
    """W[q, j] = phi_j'(x_q), by differentiating the product formula term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    W = np.zeros((len(x), n))
    for j in range(n):
        for l in range(n):
            if l == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[l]))
            for m in range(n):
                if m != j and m != l:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            W[:, j] += term
    return W


def mass_1d(k):
    """Reference 1D mass matrix B on [0, 1] (exact Gauss quadrature)."""
    nodes = gll_nodes(k)
    xq, wq = gauss_legendre(k + 1)
    V = lagrange_values(nodes, xq)
    return V.T @ (wq[:, None] * V)


def stiffness_1d(k):
    """Reference 1D stiffness matrix D on [0, 1] (exact Gauss quadrature)."""
    nodes = gll_nodes(k)
    xq, wq = gauss_legendre(k + 1)
    W = lagrange_derivatives(nodes, xq)
    return W.T @ (wq[:, None] * W)


def prolongation_1d(k, c):
    """(P_c)_ij = phi_j((xi_i + c)/2): coarse parent basis at the nodes of child c."""
    nodes = gll_nodes(k)
    return lagrange_values(nodes, 0.5 * (nodes + c))
