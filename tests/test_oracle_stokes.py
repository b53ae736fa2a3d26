"""Pins of the implicit Stokes step (paper section 2.2, spaces and forms;
section 2.3, eq. (MCS_step1), static condensation, element-wise BDDC) in the
oracle, against what the mathematics fixes:

  * the stress space: its dimension, trace-free values and nt-traces of
    degree k on interior facets (checked by a polynomial fit along the facet,
    not by the constraint functionals the oracle uses);
  * a constant field is steady: u* = u^n, sigma = gamma = 0 and u^ equal to
    its tangential components;
  * closed forms of the continuous step (u* - u^n)/dt - div(2 nu dev eps(u*)) = 0
    for fields that are eigenfunctions of the step:
      div-free modes: -div(2 nu dev eps u) = -nu lap u, factor 1/(1 + nu dt |k|^2);
      u = (sin x, 0, 0) (not div-free): -div(2 nu dev eps u) = nu |k|^2 (2 - 2/d) u,
      factor 1/(1 + (2 - 2/d) nu dt), which pins the trace-free (dev) reading;
    convergence at order k + 1 in the M norm (2D) and bounded error in 3D;
  * the direct saddle-point solve, the condensed system and the PCG with
    the element-wise BDDC all give the same (u*, u^);
  * the energy identity obtained by testing with the solution itself;
  * planted mistakes in the oracle are caught.
"""
import numpy as np
import pytest

import synth
from oracle import basis as OB
from oracle import operator as O
from oracle import stokes as ST
from oracle.space import Space


def _space(d, n, k, walls=False, lengths=None, jitter=0.0):
    per = tuple(a != 1 for a in range(d)) if walls else (True,) * d
    m = synth.kuhn_mesh(d, (n,) * d, periodic=per, lengths=lengths, jitter=jitter,
                        jitter_seed=7 if jitter else None)
    return Space(m.elem_vid, m.elem_xyz, k)


def _mrel(sp, a, b):
    M = O.mass_matrix(sp)
    e = a - b
    return float(np.sqrt(e @ M @ e / (b @ M @ b)))


def _sin_x(w, d):
    def f(x):
        z = 0.0 * x[..., 0]
        return np.stack([np.sin(w * x[..., 0])] + [z] * (d - 1), -1)
    return f


def _sin_y_wall(d):
    def f(x):
        z = 0.0 * x[..., 0]
        return np.stack([np.sin(np.pi * x[..., 1])] + [z] * (d - 1), -1)
    return f


# ------------------------------------------------------------ the spaces
@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_sigma_space_dimension_trace_and_nt_degree(d, k):
    sp = _space(d, 3, k, walls=True, jitter=0.1)
    t = sp.topo
    rng = np.random.default_rng(3)
    for T in range(min(t.n_elems, 8)):
        b = ST.element_blocks(sp, T, 1.0)
        n_int = int((t.elem_facet[T] >= 0).sum())
        assert b["N"].shape[1] == ST.expected_sigma_dim(d, k, n_int)
        sig = [rng.standard_normal(b["N"].shape[1]) if e == T else None for e in range(T + 1)]
        xr = rng.random((20, d)) / d
        val = ST.sigma_at(sp, {T: b}, sig, T, xr)
        assert np.abs(np.einsum("qii->q", val)).max() <= 1e-12 * np.abs(val).max()
        for i in range(d + 1):
            nF, tang, _, _, xv = ST.facet_frame(sp, T, i)
            # points along the facet in its own coordinates s, fit a polynomial
            # of degree k + 1 and read off its top-degree part
            ns = 40
            s = rng.random((ns, d - 1)) / (d - 1)
            o, Em, _ = OB.ref_facet_map(d, i)
            vals = ST.sigma_at(sp, {T: b}, sig, T, o[None, :] + s @ Em.T)
            mons = OB.multi_indices(d - 1, k + 1)
            V = np.stack([np.prod(s ** np.array(m), 1) for m in mons], 1)
            topm = np.array([sum(m) == k + 1 for m in mons])
            for c in range(d - 1):
                f = np.einsum("i,qij,j->q", nF, vals, tang[c])
                coef = np.linalg.lstsq(V, f, rcond=None)[0]
                assert np.abs(V @ coef - f).max() <= 1e-10 * np.abs(f).max()
                top = np.abs(coef[topm]).max() / np.abs(coef).max()
                if t.elem_facet[T, i] >= 0:
                    assert top <= 1e-9, (T, i, c, top)
                else:
                    assert top >= 1e-6, (T, i, c, top)  # wall facets keep degree k + 1


# ------------------------------------------------------------ constant field
@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (3, 1)])
def test_constant_field_is_steady(d, k):
    sp = _space(d, 3, k)
    c = np.array([0.3, -0.7, 0.45][:d])
    un = sp.interpolate(synth.constant_field(c))
    us, uh, sig, gam, bl = ST.step1(sp, un, 0.2, 0.1)
    # rounding of the sparse LU of the saddle-point system
    assert np.abs(us - un).max() <= 1e-11 * np.abs(un).max()
    assert max(np.abs(s).max() for s in sig) <= 1e-8
    assert np.abs(gam).max() <= 1e-8
    # u^ = tangential components of c: mode 0 only (psi_0 = 1 in 2D,
    # sqrt(2) in 3D on the reference facet)
    t = sp.topo
    uh = uh.reshape(t.n_facets, d - 1, sp.nf)
    psi0 = 1.0 if d == 2 else np.sqrt(2.0)
    for F in range(t.n_facets):
        T, i = t.facet_elems[F, 0], t.facet_local[F, 0]
        _, tang, _, _, _ = ST.facet_frame(sp, T, i)
        assert np.allclose(uh[F, :, 0], tang @ c / psi0, atol=1e-11, rtol=0)
        assert np.abs(uh[F, :, 1:]).max(initial=0.0) <= 1e-11


# ------------------------------------------------------------ closed forms 2D
NU, DT = 0.1, 0.1


@pytest.mark.parametrize("case", ["tg", "sinx", "wall"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_decay_factor_and_order_2d(case, k):
    w = 2 * np.pi
    if case == "tg":
        f, fac, walls = synth.taylor_green_2d(), 1 / (1 + 2 * w * w * NU * DT), False
    elif case == "sinx":
        f, fac, walls = _sin_x(w, 2), 1 / (1 + w * w * NU * DT), False
    else:
        f, fac, walls = _sin_y_wall(2), 1 / (1 + np.pi ** 2 * NU * DT), True
    errs = []
    for n in (4, 8):
        sp = _space(2, n, k, walls=walls)
        un = sp.interpolate(f)
        us = ST.step1(sp, un, NU, DT)[0]
        errs.append(_mrel(sp, us, fac * un))
    rate = np.log2(errs[0] / errs[1])
    assert rate >= (1.5 if k == 1 else k + 0.75), (errs, rate)
    assert errs[1] <= [7e-2, 5e-3, 6e-4][k - 1], errs


# ------------------------------------------------------------ closed forms 3D
@pytest.mark.parametrize("case", ["tg", "sinx", "wall"])
def test_decay_factor_3d(case):
    nu, dt = 0.5, 0.5
    L = (2 * np.pi,) * 3
    if case == "tg":
        f, fac, walls, lengths = synth.taylor_green_3d(), 1 / (1 + 3 * nu * dt), False, L
        wrong = None
    elif case == "sinx":
        # dev: factor 1/(1 + 4/3 nu dt); without the trace-free part 1/(1 + 2 nu dt)
        f, fac, walls, lengths = _sin_x(1.0, 3), 1 / (1 + 4.0 / 3.0 * nu * dt), False, L
        wrong = 1 / (1 + 2 * nu * dt)
    else:
        f, walls, lengths = _sin_y_wall(3), True, None
        nu, dt = 0.02, 0.5
        fac, wrong = 1 / (1 + np.pi ** 2 * nu * dt), None
    sp = _space(3, 3, 3 if case == "tg" else 2, walls=walls, lengths=lengths)
    un = sp.interpolate(f)
    us, _ = ST.step1_condensed(sp, un, nu, dt)
    err = _mrel(sp, us, fac * un)
    assert err <= 0.03, err
    if wrong is not None:
        assert _mrel(sp, us, wrong * un) >= 0.1


# ------------------------------------------------------------ solver routes
@pytest.mark.parametrize("d,k,n,walls", [(2, 2, 4, True), (2, 3, 3, False), (3, 1, 3, False), (3, 2, 3, True)])
def test_direct_condensed_and_pcg_agree(d, k, n, walls):
    sp = _space(d, n, k, walls=walls, jitter=0.1)
    rng = np.random.default_rng(11)
    un = sp.interpolate(_sin_y_wall(d) if walls else synth.taylor_green_2d() if d == 2
                        else synth.taylor_green_3d())
    un = un + 1e-2 * rng.standard_normal(un.shape)
    r = O.residual(sp, un, -1)
    nu, dt = 0.05, 0.02
    us, uh, sig, gam, bl = ST.step1(sp, un, nu, dt, r)
    schur = ST.schur_system(sp, nu, dt, bl)
    us2, uh2 = ST.step1_condensed(sp, un, nu, dt, r, schur)
    sc = np.abs(us).max()
    assert np.abs(us2 - us).max() <= 1e-10 * sc
    assert np.abs(uh2 - uh).max() <= 1e-10 * max(sc, np.abs(uh).max())
    us3, uh3, its = ST.step1_pcg(sp, un, nu, dt, r, rtol=1e-13, schur=schur)
    assert np.abs(us3 - us).max() <= 1e-10 * sc
    assert np.abs(uh3 - uh).max() <= 1e-10 * max(sc, np.abs(uh).max())
    assert its < 200
    # energy identity: test the step with (u*, u^, gamma) and the first
    # equation with sigma: (u* - u^n) . M u*/dt + ||sigma||^2/(2 nu) + r . u* = 0
    M = O.mass_matrix(sp)
    lhs = (us - un) @ (M @ us) / dt + ST.viscous_energy(bl, sig, nu) + r @ us
    scale = abs(un @ (M @ un)) / dt
    assert abs(lhs) <= 1e-11 * scale


def test_schur_blocks_spd_and_bddc_symmetric():
    sp = _space(2, 3, 2, walls=True, jitter=0.1)
    schur = ST.schur_system(sp, 0.05, 0.02)
    S, STb, loc, _ = schur
    for T, S_T in enumerate(STb):
        m = loc[T] >= 0
        ev = np.linalg.eigvalsh(S_T[np.ix_(m, m)])
        assert ev.min() > 0
    Sd = S.toarray()
    assert np.abs(Sd - Sd.T).max() <= 1e-12 * np.abs(Sd).max()
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal((2, S.shape[0]))
    cx, cy = ST.bddc_apply(sp, schur, x), ST.bddc_apply(sp, schur, y)
    assert abs(x @ cy - y @ cx) <= 1e-12 * abs(x @ cy)
    assert x @ cx > 0


# ------------------------------------------------------------ planted mistakes
def _sinx_error():
    sp = _space(2, 4, 2)
    un = sp.interpolate(_sin_x(2 * np.pi, 2))
    us = ST.step1(sp, un, NU, DT)[0]
    return _mrel(sp, us, un / (1 + 4 * np.pi ** 2 * NU * DT))


def _tg_error():
    sp = _space(2, 4, 2)
    un = sp.interpolate(synth.taylor_green_2d())
    us = ST.step1(sp, un, NU, DT)[0]
    return _mrel(sp, us, un / (1 + 8 * np.pi ** 2 * NU * DT))


def test_pins_pass_unmutated():
    assert _sinx_error() <= 0.02 and _tg_error() <= 0.05


def test_planted_trace_in_stress_is_caught(monkeypatch):
    orig = ST.tracefree_basis
    monkeypatch.setattr(ST, "tracefree_basis", lambda d: np.concatenate([orig(d), np.eye(d)[None]]))
    assert _sinx_error() > 0.05


def test_planted_flipped_facet_term_is_caught(monkeypatch):
    orig = ST.facet_frame

    def flipped(sp, T, i):
        nF, tang, NFn, sgn, xv = orig(sp, T, i)
        return nF, tang, NFn, -sgn, xv
    monkeypatch.setattr(ST, "facet_frame", flipped)
    assert _tg_error() > 0.05


def test_planted_missing_weak_symmetry_is_caught(monkeypatch):
    monkeypatch.setattr(ST, "skew_basis", lambda d: np.zeros((0, d, d)))
    assert _sinx_error() > 0.05 or _tg_error() > 0.05
