"""Pins of the oracle's projection step (paper section 2.3, eq. (MCS_step2),
update eq. (UpdateStep) read as u^{n+1} = u* - u~): the hybridised solve
against the same projection written without hybridisation, the pointwise
properties the paper derives (normal continuity of u~, div(u* - u~) = 0),
idempotence, and the facet pairing b3 against quadrature."""
import numpy as np
import pytest

import synth
from synth.configs import coefficient_noise
from oracle import space as S, operator as O, projection as P


def _state(cfg, n, k, noise=1e-3):
    """u* = one convection substep of a seeded state (not divergence-free)."""
    mesh, field, c = synth.make_config(cfg, n_override=n)
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    u = sp.interpolate(field, nq1d=k + 3) + coefficient_noise(cfg, sp.n_dof, noise)
    ustar = O.substep(sp, u, 0.05, k - 1)
    return sp, u, ustar


CASES = [(1, (4, 4), 2), (1, (3, 5), 3), (2, (3, 3, 3), 2), (3, (3, 2, 3), 2)]


@pytest.mark.parametrize("cfg,n,k", CASES)
def test_hybrid_equals_dense_projection(cfg, n, k):
    sp, u, ustar = _state(cfg, n, k)
    unew = P.project(sp, ustar)[0]
    ref = P.projection_dense(sp, ustar)
    scale = np.sqrt(ustar @ O.mass_apply(sp, ustar))
    e = unew - ref
    assert np.sqrt(abs(e @ O.mass_apply(sp, e))) <= 1e-11 * scale


@pytest.mark.parametrize("cfg,n,k", CASES)
def test_projection_properties(cfg, n, k):
    sp, u, ustar = _state(cfg, n, k)
    unew, ut, p, ph = P.project(sp, ustar)
    div0 = O.divergence_l2(sp, ustar)
    assert div0 > 1e-6                       # the substep broke div u = 0 ...
    assert O.divergence_l2(sp, unew) <= 1e-11 * div0 * 1e3   # ... the projection restores it
    scale = np.abs(ut).max()
    jump, wall = P.normal_jump(sp, ut)
    assert jump <= 1e-11 * scale and wall <= 1e-11 * scale   # u~ in V_h
    # idempotent, and M-orthogonal: (u_new, u~) = 0
    again = P.project(sp, unew)[0]
    sc = np.sqrt(unew @ O.mass_apply(sp, unew))
    d = again - unew
    assert np.sqrt(abs(d @ O.mass_apply(sp, d))) <= 1e-11 * sc
    ut_h = ustar - unew
    assert abs(unew @ O.mass_apply(sp, ut_h)) <= 1e-11 * sc * np.sqrt(ut_h @ O.mass_apply(sp, ut_h)) + 1e-300


def test_divergence_free_input_unchanged():
    mesh, field, c = synth.make_config(2, n_override=(3, 3, 3))
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, 2)
    u = sp.interpolate(field, nq1d=10)         # commuting interpolant: div-free
    unew = P.project(sp, u)[0]
    e = unew - u
    assert np.sqrt(abs(e @ O.mass_apply(sp, e))) <= 1e-12 * np.sqrt(u @ O.mass_apply(sp, u))


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 2)])
def test_facet_pairing_matches_quadrature(dim, k):
    # b3(phi_{T,i}, psi~_{F,j}) = int_F (phi . n_T) psi_j / |N_F| is sigma on
    # the matching facet DoF and zero otherwise
    cfg, n = (1, (3, 3)) if dim == 2 else (2, (3, 3, 3))
    mesh, field, c = synth.make_config(cfg, n_override=n)
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    t = sp.topo
    fb = np.arange(t.n_facets)
    T, T2, phiT, phiT2, nvec, ds = O._facet_traces(sp, fb)
    psi = sp.psi_q                                       # [nqf][nf]
    for side, (E_, ph, sgn) in enumerate(((T, phiT, 1.0), (T2, phiT2, -1.0))):
        nT = sgn * nvec                                  # outward for this side
        loc = t.facet_local[fb, side]
        v = np.einsum("bqid,bd,bq,qj->bji", ph, nT, ds, psi) / t.NF_norm[E_, loc][:, None, None]
        want = np.zeros_like(v)
        for b in range(len(fb)):
            s = t.sigma[E_[b], loc[b]]
            for j in range(sp.nf):
                want[b, j, loc[b] * sp.nf + j] = s
        assert np.abs(v - want).max() <= 1e-12
