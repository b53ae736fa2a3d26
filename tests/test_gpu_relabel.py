"""GPU parity on relabelled meshes: a random element order, random vertex
ids and a random local vertex order per element.  The library batches
elements by the local indices of their neighbours' facets; on the Kuhn
meshes those signatures repeat in runs, while here they mix, so the
batches are more than twice as many, every one of them padded, and the
trace-table combinations within a wave vary."""
import ctypes as C

import numpy as np
import pytest

from synth.mesh import Mesh
from oracle import space as S, operator as O
from gpu_util import case, gpu_space, dev, host, check_dual, check_mixed, check_primal

pytestmark = pytest.mark.gpu


def relabel(mesh, seed):
    rng = np.random.default_rng(seed)
    E, d = mesh.elem_vid.shape[0], mesh.dim
    perm = rng.permutation(E)
    vmap = rng.permutation(int(mesh.elem_vid.max()) + 1)
    vid = vmap[mesh.elem_vid[perm]]
    xyz = mesh.elem_xyz[perm]
    lp = np.argsort(rng.random((E, d + 1)), axis=1)
    vid = np.take_along_axis(vid, lp, 1)
    xyz = np.take_along_axis(xyz, lp[:, :, None], 1)
    return Mesh(d, np.ascontiguousarray(vid), np.ascontiguousarray(xyz))


def padded_batches(mesh):
    from paper_2408_06698_amd import _lib as L
    vid = np.ascontiguousarray(mesh.elem_vid, dtype=np.int64)
    xyz = np.ascontiguousarray(mesh.elem_xyz, dtype=np.float64)
    args = (mesh.dim, vid.shape[0], vid.ctypes.data_as(C.c_void_p), xyz.ctypes.data_as(C.c_void_p), 5)
    n = L.lib().hopu_host_mesh(*args, None, 0)
    b = np.zeros(n, dtype=np.int32)
    L.lib().hopu_host_mesh(*args, b.ctypes.data_as(C.c_void_p), n)
    b = b.reshape(-1, 16)
    return int(np.sum((b < 0).any(axis=1))), b.shape[0]


@pytest.mark.parametrize("cfg,n,k", [(2, (4, 4, 3), 3), (3, (3, 5, 3), 4)])
def test_relabelled_mesh(cfg, n, k):
    mesh0, sp0, x0, c = case(cfg, n, k, noise=1e-3)
    mesh = relabel(mesh0, 6698 + cfg)
    pad0, nb0 = padded_batches(mesh0)
    pad, nb = padded_batches(mesh)
    print(f"cfg={cfg} k={k}: padded batches {pad0}/{nb0} (Kuhn order) -> {pad}/{nb} (relabelled)")
    assert nb >= 2 * nb0 and pad == nb
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    import synth
    _, field, _ = synth.make_config(cfg, n_override=n)
    x = sp.interpolate(field, nq1d=k + 4) + 1e-3 * np.random.default_rng(5).standard_normal(sp.n_dof)
    l = k - 1
    h = gpu_space(mesh, k)
    h.set_upwind(l)
    h.set_solver(rtol=1e-13, max_it=2000)
    u = dev(x)
    r_ref = O.residual(sp, x, l)
    check_dual(sp, host(h.apply(u)), r_ref, 1e-12, "relabelled apply fp64")
    check_mixed(sp, host(h.apply(u, prec=1)), r_ref, 1e-6, "relabelled apply fp32")
    check_mixed(sp, host(h.apply(u, prec=3)), r_ref, 1e-6, "relabelled apply bf16x3")
    mu = np.random.default_rng(6).standard_normal(sp.n_dof)
    check_dual(sp, host(h.vjp(u, dev(mu))), O.vjp(sp, x, mu, l), 1e-12, "relabelled vjp fp64")
    check_mixed(sp, host(h.vjp(u, dev(mu), prec=1)), O.vjp(sp, x, mu, l), 1e-6, "relabelled vjp fp32")
    w, its = h.mass_solve(dev(r_ref), rtol=1e-13, max_it=2000)
    check_primal(sp, host(w), O.mass_solve(sp, r_ref), 1e-12, f"relabelled mass solve ({its} its)")
    steps, dt = 3, 1e-3
    h.substeps(u, dt, steps)
    check_primal(sp, host(u), O.substeps(sp, x, dt, steps, l), 1e-12, "relabelled substeps")
