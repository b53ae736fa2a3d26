"""The seeded synthetic inputs: the same seed gives the same mesh, field and
noise; the fields have the properties the recipe states (divergence-free,
periodic in the periodic directions, zero at the walls, RMS 1 for the
random curl fields); the wall grading has the stated first cell, ratio and
aspect."""
import numpy as np
import pytest

import synth
from synth import fields
from synth.configs import CONFIGS, _y_nodes, coefficient_noise, fd_directions

SMALL = {1: (4, 3), 2: (3, 3, 3), 3: (3, 4, 3), 4: (3, 3, 3), 5: (4, 4, 3)}


def _box(c):
    cfg = CONFIGS[c]
    return np.array([1.0 if L is None else L for L in cfg["lengths"]])


def _points(c, n=64, seed=0):
    L = _box(c)
    return np.random.default_rng(seed).uniform(0.05, 0.95, size=(n, len(L))) * L


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5])
def test_same_seed_same_inputs(c):
    m1, f1, _ = synth.make_config(c, n_override=SMALL[c])
    m2, f2, _ = synth.make_config(c, n_override=SMALL[c])
    assert np.array_equal(m1.elem_vid, m2.elem_vid)
    assert np.array_equal(m1.elem_xyz, m2.elem_xyz)
    x = _points(c)
    assert np.array_equal(f1(x), f2(x))
    assert np.array_equal(coefficient_noise(c, 100, 1e-3), coefficient_noise(c, 100, 1e-3))
    assert np.array_equal(fd_directions(c, 2, 50), fd_directions(c, 2, 50))


def test_jitter_is_seeded_and_optional():
    a, _, _ = synth.make_config(3, n_override=SMALL[3])
    b, _, _ = synth.make_config(3, n_override=SMALL[3], with_jitter=False)
    assert a.elem_vid.shape == b.elem_vid.shape
    assert not np.array_equal(a.elem_xyz, b.elem_xyz)


def _div(f, x, h=1e-4):
    """Fourth-order central differences of div f at the points x."""
    d = x.shape[1]
    div = np.zeros(len(x))
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        div += (-f(x + 2 * e)[:, j] + 8 * f(x + e)[:, j] - 8 * f(x - e)[:, j] + f(x - 2 * e)[:, j]) / (12 * h)
    return div


def _grad_scale(f, x, h=1e-4):
    d = x.shape[1]
    g = 0.0
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        g = max(g, np.abs((f(x + e) - f(x - e)) / (2 * h)).max())
    return g


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5])
def test_fields_divergence_free(c):
    _, f, _ = synth.make_config(c, n_override=SMALL[c])
    x = _points(c, seed=c)
    assert np.abs(_div(f, x)).max() <= 1e-9 * _grad_scale(f, x)


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5])
def test_fields_periodic(c):
    cfg = CONFIGS[c]
    _, f, _ = synth.make_config(c, n_override=SMALL[c])
    L = _box(c)
    x = _points(c, seed=10 + c)
    u = f(x)
    for j in range(cfg["dim"]):
        if cfg["periodic"][j]:
            s = np.zeros(cfg["dim"])
            s[j] = L[j]
            assert np.abs(f(x + s) - u).max() <= 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("c", [3, 5])
def test_wall_fields_vanish_at_walls_and_have_rms_one(c):
    _, f, _ = synth.make_config(c, n_override=SMALL[c])
    L = _box(c)
    x = _points(c, seed=20 + c)
    for yw in (0.0, 1.0):
        xw = x.copy()
        xw[:, 1] = yw
        assert np.abs(f(xw)).max() <= 1e-13
    # RMS over the box by a finer midpoint grid than the one that scaled it
    assert fields.field_rms(f, tuple(L), n=24) == pytest.approx(1.0, rel=2e-2)


def test_periodic_curl_field_rms_one():
    _, f, _ = synth.make_config(4, n_override=SMALL[4])
    assert fields.field_rms(f, tuple(_box(4)), n=40) == pytest.approx(1.0, rel=2e-2)


def test_coefficient_noise_level():
    e = coefficient_noise(2, 200_000, 1e-3)
    assert abs(e.mean()) <= 2e-5 and e.std() == pytest.approx(1e-3, rel=1e-2)


def test_wall_grading():
    # one-sided: first cell 1.04e-3 (aspect 20 against the 1/48 cells in x and
    # z), constant ratio 1.1, nodes exactly on [0, 1]
    y = _y_nodes(CONFIGS[3])
    d = np.diff(y)
    assert y[0] == 0.0 and y[-1] == 1.0 and len(d) == 48
    assert np.allclose(d[1:] / d[:-1], 1.1, rtol=1e-12)
    assert (1.0 / 48) / d[0] == pytest.approx(20.0, rel=1e-3)
    # symmetric: finest cells at both walls, aspect 50 against dx = 4/96
    y = _y_nodes(CONFIGS[5])
    d = np.diff(y)
    assert len(d) == 64 and abs(y[-1] - 1.0) <= 1e-15
    assert np.allclose(d, d[::-1], rtol=1e-12)
    assert d.min() == d[0] and (4.0 / 96) / d[0] == pytest.approx(50.0, rel=1e-3)
