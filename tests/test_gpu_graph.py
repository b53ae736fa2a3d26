"""The convection apply under HIP graph capture.  hopu_convection_apply
launches its kernels on the context's stream and makes no allocation, copy,
memset or synchronisation, so a caller can capture it into a graph (for the
launch-bound small workloads).  Each replay is checked against the eager
apply of the state the graph reads at that moment, with eager work and
synchronisations between the replays."""
import numpy as np
import pytest
import torch

from gpu_util import case, dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,n,k", [(1, (16, 16), 2), (2, (4, 3, 3), 3), (3, (3, 3, 4), 5)])
def test_apply_graph_replays_match_eager(cfg, n, k):
    from paper_2408_06698_amd import FP64, FP32_MFMA
    from paper_2408_06698_amd.hopu import Hopu
    mesh, sp, x, c = case(cfg, n, k, noise=1e-3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = Hopu(mesh.dim, k, mesh.elem_vid, mesh.elem_xyz, stream=s)
        h.set_upwind(k - 1)
        u = dev(x)
        r_graph = h.zeros()
        r32_graph = h.zeros()
        h.apply(u, r_graph)                      # warm-up outside the capture
        h.apply(u, r32_graph, prec=FP32_MFMA)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h.apply(u, r_graph)
        h.apply(u, r32_graph, prec=FP32_MFMA)
    rng = np.random.default_rng(cfg)
    for rep in range(3):
        xr = x * (1.0 + 0.1 * rep) + 1e-3 * rng.standard_normal(x.shape)
        with torch.cuda.stream(s):
            u.copy_(dev(xr))
            want = h.apply(u)                    # eager, on the same stream
            want32 = h.apply(u, prec=FP32_MFMA)
        s.synchronize()
        g.replay()
        s.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(r_graph, want), (cfg, rep)
        assert torch.equal(r32_graph, want32), (cfg, rep)
    h.close()
