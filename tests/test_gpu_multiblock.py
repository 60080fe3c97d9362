"""GPU parity of the multi-block DSS (Sec. 4.3, Algorithm 8) against the oracle's
S = G G^T with a global numbering from node positions: the structured cascade
per block plus the macro-face pairs and the macro-line and macro-vertex
gather-scatter passes must give every copy the sum of all copies of its node,
bit for bit on integer data (any order of exact sums), to rounding on random
data, and the averaging version must be the projection S_bar."""
import numpy as np
import pytest
import torch

from oracle.multiblock import MultiBlockMesh
from synthetic_inputs import integer_valued, uniform

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,n", [(1, 1), (1, 3), (2, 2), (3, 2), (4, 3), (7, 1)])
def test_multiblock_dss_matches_the_oracle(gpu_lib, k, n):
    fe = gpu_lib
    print("multiblock", k, n, flush=True)
    M = MultiBlockMesh(k, n)
    G = fe.MultiBlock(k, n)
    assert G.len == M.len and G.n_nodes == M.n_nodes
    c = G.counts()
    m = k * n
    # macro-lines: 12 centre edges + 8 diagonals (valence 3) and 12 outer edges (valence 2),
    # m - 1 DoFs each; macro-vertices: 8 inner + 8 outer corners
    assert c["line_dofs"] == 32 * (m - 1) and c["vertex_dofs"] == 16
    v = integer_valued(M.len, seed=300 + k)
    vd = torch.as_tensor(v, device="cuda")
    G.dss(vd)
    torch.cuda.synchronize()
    assert np.array_equal(vd.cpu().numpy(), M.dss(v))
    for dtype, tol in ((torch.float64, 1e-15), (torch.float32, 1e-6)):
        w = uniform(M.len, seed=310 + k)
        wd = torch.as_tensor(w, dtype=dtype, device="cuda")
        G.dss(wd)
        ref = M.dss(w)
        got = wd.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref)) <= tol * 8 * np.max(np.abs(ref)), dtype
        wa = torch.as_tensor(w, dtype=dtype, device="cuda")
        G.dss(wa, averaging=True)
        refa = M.dss_average(w)
        assert np.max(np.abs(wa.cpu().numpy() - refa)) <= tol * 8 * np.max(np.abs(refa)), dtype
    # continuous vectors are fixed points of the averaging DSS
    x = M.G @ uniform(M.n_nodes, seed=320)
    xd = torch.as_tensor(x, device="cuda")
    G.dss(xd, averaging=True)
    assert np.max(np.abs(xd.cpu().numpy() - x)) < 1e-15 * np.max(np.abs(x)) * 4
    G.close()


def test_multiblock_rejects_oversize(gpu_lib):
    fe = gpu_lib
    with pytest.raises(fe.FeError):
        fe.MultiBlock(8, 256)
