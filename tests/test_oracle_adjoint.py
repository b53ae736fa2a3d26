"""Pins of the oracle's transpose Jacobian against a dense Jacobian
assembled independently by double loops over physical basis products
(the linearisation of the HOPU residual of section 3.2, eq.
(hopudefinition), in conservative volume form), on the two-element meshes
and on a periodic 4x4 mesh of the 2D Taylor-Green workload.

The assembled J(w) is itself pinned by two facts that do not depend on
either code: r is homogeneous of degree 2, so J(w) w = 2 r(w) exactly, and
J(w) d equals the central difference of r along d (r is piecewise
quadratic in u, so the difference is exact up to rounding unless a
quadrature point's u.n changes sign inside [w - h d, w + h d])."""
import numpy as np
import pytest

import synth
from synth.mesh import two_element_mesh
from oracle import space as S, operator as O


def _check_jacobian(sp, w, l, seed, fd_dirs=3):
    rng = np.random.default_rng(seed)
    Jm = O.assemble_jacobian(sp, w, l)
    r = O.residual(sp, w, l)
    scale = np.abs(Jm).max() * np.abs(w).max()
    # homogeneity: J(w) w = 2 r(w)
    assert np.abs(Jm @ w - 2.0 * r).max() <= 1e-13 * scale
    # central differences of r
    h = 1e-6
    for _ in range(fd_dirs):
        d = rng.standard_normal(sp.n_dof)
        fd = (O.residual(sp, w + h * d, l) - O.residual(sp, w - h * d, l)) / (2 * h)
        jd = Jm @ d
        assert np.abs(fd - jd).max() <= 1e-7 * np.abs(jd).max()
    # the matrix-free transpose Jacobian against the assembled transpose
    for _ in range(3):
        mu = rng.standard_normal(sp.n_dof)
        g = O.vjp(sp, w, mu, l)
        want = Jm.T @ mu
        assert np.abs(g - want).max() <= 1e-13 * np.abs(Jm).max() * np.abs(mu).max()
    return Jm


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 1), (3, 2)])
def test_assembled_jacobian_two_elements(dim, k):
    """(The 2D k = 1 pair is left out: its two DoFs span only fields whose
    residual cancels to rounding, so every check there is vacuous.)"""
    m = two_element_mesh(dim)
    sp = S.Space(m.elem_vid, m.elem_xyz, k)
    w = np.random.default_rng(100 + 10 * dim + k).standard_normal(sp.n_dof)
    for l in (-1, 0, k - 1, k):
        _check_jacobian(sp, w, l, seed=dim * 100 + k * 10 + l + 1)


def test_assembled_jacobian_periodic_c1_mesh():
    """4x4 periodic mesh of the 2D Taylor-Green recipe, k = 2, l = 1, at the
    noisy Taylor-Green state (every facet has both neighbours)."""
    m, f, cfg = synth.make_config(1, n_override=(4, 4))
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    w = sp.interpolate(f, nq1d=10) + 1e-3 * np.random.default_rng(5).standard_normal(sp.n_dof)
    _check_jacobian(sp, w, 1, seed=41)


def test_jacobian_at_zero_normal_velocity():
    """A state with u.n = 0 on every facet between rows (the layered flow
    with c = 0: u = (p(y), 0), one constant per row of cells) has tangential
    jumps exactly where u.n vanishes, the case of the reading sgn(0) = 0:
    the assembled Jacobian and the transpose Jacobian still agree."""
    from synth.mesh import kuhn_mesh
    mesh = kuhn_mesh(2, (3, 4), (1.0, 1.0), (True, True))
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, 2)
    p = np.array([0.3, -0.7, 1.1, 0.2])

    def f(x):
        row = np.floor(x[..., 1] * 4 + 1e-9).astype(int) % 4
        return np.stack([p[row], 0.0 * x[..., 0]], -1)

    w = sp.interpolate(f)
    Jm = O.assemble_jacobian(sp, w, -1)
    rng = np.random.default_rng(3)
    for _ in range(3):
        mu = rng.standard_normal(sp.n_dof)
        assert np.abs(O.vjp(sp, w, mu, -1) - Jm.T @ mu).max() <= 1e-13 * np.abs(Jm).max() * np.abs(mu).max()


def test_dropped_sign_term_is_caught(monkeypatch):
    """A planted mistake in the adjoint (the 1/2 sgn(u.n) term of s
    dropped) breaks the assembled-transpose pin."""
    m = two_element_mesh(2)
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    w = np.random.default_rng(7).standard_normal(sp.n_dof)
    Jm = O.assemble_jacobian(sp, w, 0)
    mu = np.random.default_rng(8).standard_normal(sp.n_dof)
    good = O.vjp(sp, w, mu, 0)
    assert np.abs(good - Jm.T @ mu).max() <= 1e-13 * np.abs(Jm).max() * np.abs(mu).max()

    class NoSign:
        def __getattr__(self, name):
            return getattr(np, name)

        @staticmethod
        def sign(v):
            return 0.0 * np.sign(v)

    monkeypatch.setattr(O, "np", NoSign())
    bad = O.vjp(sp, w, mu, 0)
    monkeypatch.undo()
    assert np.abs(bad - Jm.T @ mu).max() > 1e-6 * np.abs(Jm).max() * np.abs(mu).max()
