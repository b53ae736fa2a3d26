"""Planted mistakes in the oracle (on the CPU only) must each break a pin.
This checks that the pins can see plausible errors: a flipped normal, a
wrong projection degree, a transposed Jacobian, a dropped facet scaling, a
doubled upwind weight."""
import numpy as np
import pytest

import synth
from synth import fields
from synth.mesh import kuhn_mesh
from oracle import space as S, operator as O

VOL, CEN, UP = O.TERM_VOLUME, O.TERM_CENTRAL, O.TERM_UPWIND


def _space():
    m, f, c = synth.make_config(1, n_override=(4, 4))
    return S.Space(m.elem_vid, m.elem_xyz, 2), f


def _constant_zero_ok(sp):
    x = sp.interpolate(fields.constant_field([0.3, -0.7]))
    r = O.residual(sp, x, 1)
    rv = O.residual(sp, x, 1, VOL)
    return np.abs(r).max() <= 1e-12 * np.abs(rv).max()


def _central_energy_ok(sp, f):
    x = sp.interpolate(f, nq1d=10)
    r = O.residual(sp, x, sp.k)
    return abs(x @ r) <= 1e-11 * np.abs(r).max() * np.abs(x).max()


def test_pins_pass_unmutated():
    sp, f = _space()
    assert _constant_zero_ok(sp) and _central_energy_ok(sp, f)


def test_flipped_normal_is_caught():
    sp, f = _space()
    sp.topo.sigma = -sp.topo.sigma
    assert not _constant_zero_ok(sp)


def test_transposed_jacobian_is_caught():
    sp, f = _space()
    sp.Jinv = np.transpose(sp.Jinv, (0, 2, 1))
    assert not (_constant_zero_ok(sp) and _central_energy_ok(sp, f))


def test_wrong_projection_degree_is_caught(monkeypatch):
    sp, f = _space()
    orig = O._projector
    monkeypatch.setattr(O, "_projector", lambda s, lf: orig(s, lf - 1))
    assert not _central_energy_ok(sp, f)


def test_dropped_facet_scaling_is_caught():
    sp, f = _space()
    nf = sp.nf
    sp.S[:, :3 * nf] = 1.0
    x = sp.interpolate(fields.constant_field([0.3, -0.7]))
    # the interpolant still uses the true functionals; the basis no longer
    # reproduces the constant, so the zero pin fails
    r = O.residual(sp, x, 1)
    assert np.abs(r).max() > 1e-8


def _layered_dissipation_ok():
    """The closed-form upwind dissipation of the layered flow u = (p(y), c)
    (one constant per row of cells): 1/2 |c| sum_j (p_j - p_{j+1})^2."""
    mesh = kuhn_mesh(2, (3, 4), (1.0, 1.0), (True, True))
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, 2)
    p, c = np.array([0.3, -0.7, 1.1, 0.2]), -0.6

    def f(x):
        row = np.floor(x[..., 1] * 4 + 1e-9).astype(int) % 4
        return np.stack([p[row], np.full(x.shape[:-1], c)], -1)

    x = sp.interpolate(f)
    D = 0.5 * abs(c) * np.sum((p - np.roll(p, -1)) ** 2)
    # the identity u.r(u) = D holds with or without the mistake below; only
    # the closed form sees it
    return abs(x @ O.residual(sp, x, -1) - O.dissipation(sp, x, -1)) <= 1e-11 * D, \
        abs(O.dissipation(sp, x, -1) - D) <= 1e-12 * D


def test_doubled_upwind_weight_is_caught(monkeypatch):
    assert _layered_dissipation_ok() == (True, True)

    class DoubledAbs:
        """numpy with |.| doubled: the upwind weight 1/2 |u.n| becomes |u.n|"""
        def __getattr__(self, name):
            return getattr(np, name)

        @staticmethod
        def abs(v):
            return 2.0 * np.abs(v)

    monkeypatch.setattr(O, "np", DoubledAbs())
    assert _layered_dissipation_ok() == (True, False)


def _divergence_ok():
    from test_oracle_pins import walled_parabola_case
    sp, x, want, _ = walled_parabola_case(3, 2)
    return abs(O.divergence_l2(sp, x) - want) <= 1e-13 * want


class _NumpyWith:
    """numpy with one function replaced (a planted mistake)"""
    def __init__(self, **repl):
        self.repl = repl

    def __getattr__(self, name):
        return self.repl.get(name, getattr(np, name))


def test_divergence_mistakes_are_caught(monkeypatch):
    """The closed-form divergence pin sees a dropped |det J| weight, a
    missing square root and a doubled value."""
    assert _divergence_ok()
    monkeypatch.setattr(O, "np", _NumpyWith(abs=lambda v: np.ones_like(np.abs(v))))
    assert not _divergence_ok()
    monkeypatch.setattr(O, "np", _NumpyWith(sqrt=lambda v: v))
    assert not _divergence_ok()
    monkeypatch.setattr(O, "np", _NumpyWith(sqrt=lambda v: 2.0 * np.sqrt(v)))
    assert not _divergence_ok()
