"""Writes coef_scale.json: the coefficient scale s = 1 / max |g| over every
Gauss point of the finest mesh (the reading of the workload's
exp(U[-1, 1] smooth field)) for the deformed benchmark meshes, computed by the
oracle alone (oracle.geometry.coefficient_scale), so that GPU tests at those
sizes can build the oracle geometry of a cell subset without recomputing it.

    python tests/golden/make_coef_scale.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.geometry import coefficient_scale  # noqa: E402
from oracle.mesh import StructuredMesh  # noqa: E402
from synthetic_inputs import coefficient_modes  # noqa: E402

CASES = [(3, 48, 0.1, 2), (7, 64, 0.1, 2)]


def main():
    out = {"_source": "oracle.geometry.coefficient_scale on the finest mesh; key k_n_amp_seed",
           "scales": {}}
    for k, n, amp, seed in CASES:
        t0 = time.time()
        s = coefficient_scale(StructuredMesh(3, k, n), amp, coefficient_modes(seed), chunk=512)
        out["scales"]["%d_%d_%g_%d" % (k, n, amp, seed)] = s
        print("k=%d n=%d: scale %.17g (%.1f s)" % (k, n, s, time.time() - t0), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "coef_scale.json"), "w") as f:
        json.dump(out, f, indent=2)


if __name__ == "__main__":
    main()
