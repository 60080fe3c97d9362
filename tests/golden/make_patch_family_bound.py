"""Writes patch_family_bound.json: how many MG-PCG iterations the vertex-patch
smoother needs on small deformed meshes when each patch solve is exact (dense
Cholesky of R_p A R_p^T), the best Kronecker-sum fit of each patch (the
learned model's training target), or the averaged-geometry separable factors.

Computed by the oracle alone, as a reference: the exact patch solve bounds
what any per-patch factors, learned or not, can reach with this smoother.
Setting: V-cycle (Algorithm 1) on every level of a uniform hierarchy, one
Chebyshev(3) pre- and post-smoothing step preconditioned by the patch solve,
lambda_max = 1.2 x the largest eigenvalue of P A (ARPACK), PCG to a 1e-10
relative residual from x = 0, right-hand side the seeded uniform vector.

    python tests/golden/make_patch_family_bound.py
"""
import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.geometry import DeformedGeometry, coefficient_scale  # noqa: E402
from oracle.learned import fit_targets, weights_from_targets  # noqa: E402
from oracle.mesh import StructuredMesh  # noqa: E402
from oracle.multigrid import Hierarchy, chebyshev_sweep, pcg, vcycle  # noqa: E402
from oracle.patch import patch_dof_indices  # noqa: E402
from oracle.sepfit import averaged_weights, sep_matrix  # noqa: E402
from synthetic_inputs import coefficient_modes, uniform  # noqa: E402

CASES = [  # (k, n, deformation amplitude, coefficient seed)
    (2, 8, 0.1, 2), (3, 8, 0.1, 2), (2, 8, 0.13, 1002), (3, 8, 0.13, 1002), (3, 8, 0.13, 7),
]


def patch_solvers(lev, geom, kind):
    """Dense inverses of the patch operators of one level, per patch."""
    idx = patch_dof_indices(lev.mesh)
    if kind == "exact":
        mats = [lev.A_full[i][:, i].toarray() for i in idx]
    else:
        if kind == "averaged":
            w = averaged_weights(geom)
        else:
            w = weights_from_targets(fit_targets(geom, lev.A_full, sweeps=30), lev.mesh.h)
        mats = [sep_matrix(lev.mesh.k, wp) for wp in w]
    return idx, [sla.cho_solve(sla.cho_factor(a), np.eye(a.shape[0])) for a in mats]


def make_precond(lev, idx, inv):
    def apply(r_int):
        r = lev.to_full(r_int)
        z = np.zeros_like(r)
        for i, ai in zip(idx, inv):
            z[i] += ai @ r[i]
        return lev.to_int(z)
    return apply


def run_case(k, n, amp, seed):
    coef = coefficient_modes(seed)
    scale = coefficient_scale(StructuredMesh(3, k, n), amp, coef)
    geoms = {}

    def elem_fn(m):
        geoms[m] = DeformedGeometry(StructuredMesh(3, k, m), amp, coef, scale=scale)
        return geoms[m].element_matrices()

    h = Hierarchy(3, k, n, elem_fn=elem_fn)
    b = uniform(h.levels[-1].n_int, seed=91)
    out = {}
    for kind in ("averaged", "best_fit", "exact"):
        pre, lmax = [None], [1.0]
        for l in range(1, len(h.levels)):
            lev = h.levels[l]
            idx, inv = patch_solvers(lev, geoms[h.ns[l]], kind)
            P = make_precond(lev, idx, inv)
            op = spla.LinearOperator((lev.n_int, lev.n_int), matvec=lambda v, P=P, A=lev.A: P(A @ v))
            lam = float(np.max(np.real(spla.eigs(op, k=1, which="LM", tol=1e-6,
                                                 v0=np.ones(lev.n_int), return_eigenvectors=False))))
            pre.append(P)
            lmax.append(1.2 * lam)
        def smoother(lev, l, bb, u, is_pre):
            return chebyshev_sweep(lev, bb, u, lmax[l], 3, precond=pre[l], u_is_zero=is_pre)

        _, its, hist = pcg(h.levels[-1].A, b, lambda r: vcycle(h, r, smoother), tol=1e-10)
        out[kind] = {"iterations": int(its), "lambda_max_finest": lmax[-1] / 1.2}
    return out


def main():
    res = {"_source": __doc__.strip().splitlines()[0], "cases": []}
    for k, n, amp, seed in CASES:
        t0 = time.time()
        r = run_case(k, n, amp, seed)
        res["cases"].append({"k": k, "n": n, "amp": amp, "seed": seed, **r})
        print(k, n, amp, seed, {kk: v["iterations"] for kk, v in r.items()}, "%.0f s" % (time.time() - t0), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "patch_family_bound.json"), "w") as f:
        json.dump(res, f, indent=2)


if __name__ == "__main__":
    main()
