"""Planted mistakes in the oracle (on the CPU only) must each break a pin.
This checks that the pins can see plausible errors: a flipped normal, a
wrong projection degree, a transposed Jacobian, a dropped facet scaling."""
import numpy as np
import pytest

import synth
from synth import fields
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
