"""The allocation-free evaluation entry point (hopu_eval_noalloc), through
the C ABI, against hopu_eval: two calls in a row, the second with fewer
points (the scratch keeps the first call's table; the second must not read
past its own), and the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2408_06698_amd import _lib as L
from gpu_util import case, gpu_space, dev, host

pytestmark = pytest.mark.gpu


def _eval(fn, h, u, pts):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = torch.zeros((h.n_elems, pts.shape[0], h.dim), dtype=torch.float64, device="cuda:0")
    st = fn(h.h, C.c_void_p(u.data_ptr()), pts.shape[0], pts.ctypes.data_as(C.c_void_p), C.c_void_p(out.data_ptr()))
    return st, out


@pytest.mark.parametrize("cfg,n,k", [(3, (3, 4, 3), 5), (1, (6, 5), 2)])
def test_eval_noalloc_matches_eval(cfg, n, k):
    mesh, sp, x, c = case(cfg, n, k, noise=1e-3)
    h = gpu_space(mesh, k)
    u = dev(x)
    lib = L.lib()
    rng = np.random.default_rng(5)
    d = mesh.dim
    for npts in (40, 7):  # the second call smaller than the first
        pts = rng.uniform(0, 1.0 / (d + 1), (npts, d))
        st0, ref = _eval(lib.hopu_eval, h, u, pts)
        st1, got = _eval(lib.hopu_eval_noalloc, h, u, pts)
        assert st0 == L.HOPU_OK and st1 == L.HOPU_OK
        r, g = host(ref), host(got)
        print(f"eval_noalloc cfg={cfg} k={k} n_pts={npts}: max |diff| {np.abs(r - g).max():.1e}")
        assert np.array_equal(r, g)
        # and the values are the oracle's
        vr = sp.evaluate(x, np.arange(sp.topo.n_elems), pts)
        assert np.abs(g - vr).max() <= 1e-13 * np.abs(vr).max()
    # beyond the scratch: refused with the limit in the message, nothing written
    big = rng.uniform(0, 0.2, (131072 // (h.n_loc * d) + 1, d))
    st, out = _eval(lib.hopu_eval_noalloc, h, u, big)
    assert st == L.HOPU_EINVAL
    assert "scratch" in lib.hopu_last_error(h.h).decode()
    assert not host(out).any()
    h.close()
