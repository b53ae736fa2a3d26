"""Parity at the workloads' full sizes, in the launch configuration the bench
uses: the library runs on the whole mesh; the oracle evaluates the rows of a
seeded sample of elements (their interior DoFs and the DoFs of their facets)
from the element patch around them."""
import time
import numpy as np
import pytest
import torch

import synth
from oracle import space as S, operator as O
from gpu_util import gpu_space, dev, host

pytestmark = pytest.mark.gpu


def _setup(cfg):
    t0 = time.time()
    mesh, field, c = synth.make_config(cfg)
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, c["k"])
    rng = np.random.default_rng(6698 + cfg + 2000)
    x = rng.standard_normal(sp.n_dof)
    samp = np.sort(rng.choice(sp.topo.n_elems, size=48, replace=False))
    nb = sp.topo.nbr[samp].ravel()
    patch = np.unique(np.concatenate([samp, nb[nb >= 0]]))
    g = sp.gdof[samp]
    nfl = (sp.dim + 1) * sp.nf
    rows_f = np.unique(g[:, :nfl][g[:, :nfl] >= 0])
    rows_i = np.unique(g[:, nfl:])
    print(f"cfg {cfg}: {sp.topo.n_elems} elements, {sp.n_dof} DoFs, oracle setup {time.time() - t0:.1f}s")
    return mesh, sp, x, c, patch, rows_f, rows_i


def _check(r, ref, rows_f, rows_i, tol, what):
    for name, rows in (("facet", rows_f), ("interior", rows_i)):
        e = np.linalg.norm(r[rows] - ref[rows]) / np.linalg.norm(ref[rows])
        print(f"{what} {name} rows: rel l2 {e:.2e}")
        assert e <= tol, (what, name, e)


@pytest.mark.parametrize("cfg", [2, 3])
def test_fullsize_apply_vjp_mass(cfg):
    mesh, sp, x, c, patch, rows_f, rows_i = _setup(cfg)
    k, l = c["k"], c["l"]
    h = gpu_space(mesh, k)
    h.set_upwind(l)
    u = dev(x)
    ref = O.residual(sp, x, l, elems=patch)
    _check(host(h.apply(u)), ref, rows_f, rows_i, 1e-12, "apply fp64")
    _check(host(h.apply(u, prec=1)), ref, rows_f, rows_i, 1e-5, "apply fp32")
    _check(host(h.apply(u, prec=2)), ref, rows_f, rows_i, 3e-3, "apply bf16x2")
    _check(host(h.apply(u, prec=3)), ref, rows_f, rows_i, 1e-5, "apply bf16x3")
    mu = np.random.default_rng(7).standard_normal(sp.n_dof)
    gref = O.vjp(sp, x, mu, l, elems=patch)
    _check(host(h.vjp(u, dev(mu))), gref, rows_f, rows_i, 1e-12, "vjp fp64")
    # mass rows of the sample: M restricted to the patch elements
    t = sp.topo
    y = np.zeros(sp.n_dof)
    for eb in np.array_split(patch, max(1, len(patch) // 64)):
        phi = sp.phys_vals(eb, sp.ref_vals)
        wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
        sp.scatter(y, eb, np.einsum("bq,bqid,bqjd,bj->bi", wdx, phi, phi, sp.local(x, eb)))
    _check(host(h.mass_apply(u)), y, rows_f, rows_i, 1e-13, "mass")


def test_fullsize_channel_k5_apply():
    """Workload 5 (1,769,472 tets, k = 5, 222.8M DoFs) at full size."""
    mesh, sp, x, c, patch, rows_f, rows_i = _setup(5)
    h = gpu_space(mesh, c["k"])
    h.set_upwind(c["l"])
    u = dev(x)
    ref = O.residual(sp, x, c["l"], elems=patch)
    _check(host(h.apply(u)), ref, rows_f, rows_i, 1e-12, "apply fp64 k5")
    _check(host(h.apply(u, prec=1)), ref, rows_f, rows_i, 1e-5, "apply fp32 k5")
    _check(host(h.apply(u, prec=3)), ref, rows_f, rows_i, 1e-5, "apply bf16x3 k5")


def test_fullsize_projection_properties():
    # 3D periodic Taylor-Green at the bench size (32^3 x 6 tets, k = 3): the
    # oracle's direct solve does not fit, so check what the projection must
    # satisfy at any size: u_new is divergence-free, u~ = u* - u_new is
    # M-orthogonal to u_new, and projecting again changes nothing
    from synth.configs import coefficient_noise
    mesh, field, c = synth.make_config(2)
    k = c["k"]
    h = gpu_space(mesh, k)
    u = h.interpolate(field, n1d=k + 2)
    u += torch.tensor(coefficient_noise(2, h.n_dof, c["noise"]), device=u.device)
    h.set_upwind(c["l"])
    h.substeps(u, 0.05, 1)                         # breaks div u = 0
    unew, its = h.project(u, rtol=1e-13)
    _, div0, _ = h.diagnostics(u)
    _, div1, _ = h.diagnostics(unew)
    ut = u - unew
    mu, mt = torch.sqrt(torch.dot(unew, h.mass_apply(unew))), torch.sqrt(torch.dot(ut, h.mass_apply(ut)))
    orth = float(torch.dot(unew, h.mass_apply(ut)) / (mu * mt))
    again, its2 = h.project(unew, rtol=1e-13)
    d = again - unew
    rel2 = float(torch.sqrt(torch.dot(d, h.mass_apply(d))) / mu)
    print(f"projection C2: {its} CG its, div {div0:.3e} -> {div1:.3e}, (u_new, u~)_M {orth:.1e}, "
          f"reprojection {rel2:.1e} ({its2} its)")
    assert div1 <= 1e-12 * div0
    assert abs(orth) <= 1e-10
    assert rel2 <= 1e-11
