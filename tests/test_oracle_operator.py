"""Pins of the oracle's convection operator, mass solve, substeps and
adjoints against identities implied by the paper's definitions (HOPU form,
eq. (hopudefinition); standard upwind, eq. (upwind); explicit substep of
eq. (MCS_step1); mass matrix M_uu = M / dt)."""
import math
import os

import numpy as np
import pytest
from scipy.linalg import null_space

import synth
from synth.mesh import kuhn_mesh, two_element_mesh
from synth import fields
from oracle import basis as B, quadrature as Q, space as S, operator as O

VOL, CEN, UP = O.TERM_VOLUME, O.TERM_CENTRAL, O.TERM_UPWIND


def minv_norm(sp, v):
    return math.sqrt(max(float(v @ O.mass_solve(sp, v)), 0.0))


def m_norm(sp, x):
    return math.sqrt(max(float(x @ O.mass_apply(sp, x)), 0.0))


def divfree_random(sp, seed, n_vec=None):
    """A random divergence-free element of V_h: null space of the map to the
    P^{k-1} moments of div u (div V_h lies in P^{k-1} on affine elements)."""
    t = sp.topo
    d = sp.dim
    kk = sp.k - 1
    x, w = Q.simplex_rule(d, sp.k + 1)
    qv, _ = B.scalar_basis(d, kk, x)
    rows = []
    Bm = np.zeros((t.n_elems * qv.shape[1], sp.n_dof))
    for e in range(t.n_elems):
        gphi = sp.phys_grads(np.array([e]), B.dual_basis(d, sp.k, x)[1])[0]
        div = np.einsum("qiaa->qi", gphi)  # [nq][n]
        blk = (qv * w[:, None]).T @ div      # [nPk-1][n]
        g = sp.gdof[e]
        for a in range(sp.n):
            if g[a] >= 0:
                Bm[e * qv.shape[1]:(e + 1) * qv.shape[1], g[a]] += blk[:, a]
    Nsp = null_space(Bm)
    rng = np.random.default_rng(seed)
    return Nsp @ rng.standard_normal(Nsp.shape[1])


@pytest.fixture(scope="module")
def periodic2d():
    m, f, c = synth.make_config(1, n_override=(4, 4))
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    return sp, f


@pytest.fixture(scope="module")
def periodic3d():
    m, f, c = synth.make_config(4, n_override=(3, 3, 3))
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    return sp, f


@pytest.fixture(scope="module")
def wall3d():
    m, f, c = synth.make_config(3, n_override=(3, 4, 3))
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    return sp, f


# --------------------------------------------------------------- zeros
@pytest.mark.parametrize("which", ["periodic2d", "periodic3d"])
def test_constant_field_gives_zero(which, request):
    sp, _ = request.getfixturevalue(which)
    c = np.array([0.3, -0.7, 0.45])[:sp.dim]
    x = sp.interpolate(fields.constant_field(c))
    rv = O.residual(sp, x, 1, VOL)
    rf = O.residual(sp, x, 1, CEN | UP)
    scale = minv_norm(sp, rv) + minv_norm(sp, rf)
    assert scale > 1e-3
    assert minv_norm(sp, rv + rf) <= 1e-13 * scale


def test_shear_field_on_wall_mesh_gives_zero(wall3d):
    """u = (p(y), 0, q(y)), deg <= k, on a box with walls at y = 0, 1:
    (u.grad)u = 0, div u = 0, no jumps, u.n = 0 on walls."""
    sp, _ = wall3d
    f = fields.shear_field([0.2, 1.0, -0.8], [0.1, -0.5, 0.3])
    x = sp.interpolate(f)
    rv = O.residual(sp, x, 0, VOL)
    rf = O.residual(sp, x, 0, CEN | UP)
    scale = minv_norm(sp, rv) + minv_norm(sp, rf)
    assert minv_norm(sp, rv + rf) <= 1e-13 * max(scale, 1.0)


# ------------------------------------------------- forms and skew symmetry
@pytest.mark.parametrize("which,nq", [("periodic2d", 10), ("periodic3d", 12)])
def test_advective_equals_conservative_on_divfree(which, nq, request):
    sp, f = request.getfixturevalue(which)
    x = sp.interpolate(f, nq1d=nq)
    assert O.divergence_l2(sp, x) < 1e-11 * m_norm(sp, x)
    for l in (-1, 0, sp.k):
        a = O.residual_advective(sp, x, l)
        c = O.residual(sp, x, l)
        assert minv_norm(sp, a - c) <= 1e-11 * minv_norm(sp, c)


@pytest.mark.parametrize("which", ["periodic3d", "wall3d"])
def test_conservative_equals_advective_plus_divergence_term(which, request):
    """Integration by parts on each element, for any u with continuous
    normal component (divergence-free or not): the conservative form equals
    the advective form of eq. (hopudefinition) plus int (div u)(u . phi);
    the rules integrate both exactly, so the two agree to rounding."""
    sp = request.getfixturevalue(which)[0]
    x = np.random.default_rng(11).standard_normal(sp.n_dof)
    t = sp.topo
    dterm = np.zeros(sp.n_dof)
    for eb in sp.batches(t.n_elems, sp.elem_batch_size()):
        xl = sp.local(x, eb)
        phi = sp.phys_vals(eb, sp.ref_vals)
        gphi = sp.phys_grads(eb, sp.ref_grads)
        u = np.einsum("bqid,bi->bqd", phi, xl)
        div = np.einsum("bqiaa,bi->bq", gphi, xl)
        wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
        sp.scatter(dterm, eb, np.einsum("bq,bq,bqa,bqia->bi", wdx, div, u, phi))
    assert minv_norm(sp, dterm) > 1e-2 * minv_norm(sp, O.residual(sp, x, 1))   # not divergence-free
    for l in (-1, 1, sp.k):
        c = O.residual(sp, x, l)
        a = O.residual_advective(sp, x, l)
        assert minv_norm(sp, c - (a + dterm)) <= 1e-12 * minv_norm(sp, c)


@pytest.mark.parametrize("dim", [2, 3])
def test_central_part_skew_symmetric(dim):
    m = two_element_mesh(dim)
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    w = divfree_random(sp, 7)
    A = O.assemble_picard(sp, w, -1, VOL | CEN)
    assert np.abs(A + A.T).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_upwind_dissipation_closed_form_layered_flow(dim, k):
    """u = (p(y), c) in 2D, (p(y), c, q(y)) in 3D, with p, q constant on
    each row of cells of a periodic Kuhn mesh, lies in V_h (u.n is +-c on
    the facets between rows and is taken inside one row on all others) and
    is exactly divergence-free; its only jumps are tangential,
    (p_j - p_{j+1}, 0, q_j - q_{j+1}) on the facets between rows j and j+1,
    where |u.n| = |c|.  The standard upwind flux (eq. (upwind), l = -1)
    then dissipates D = 1/2 |c| A sum_j |jump_j|^2 (rows wrap; A the area of
    one row interface), and u.r(u) = D because grad u = 0 in every element
    and the central form is skew.  For l >= 0 the jump is a constant on
    each facet, which Pi^l keeps, so nothing is dissipated."""
    ny = 4
    n = (3, ny) if dim == 2 else (3, ny, 3)
    lengths = (1.0, 1.0) if dim == 2 else (1.5, 1.0, 0.5)
    mesh = kuhn_mesh(dim, n, lengths, (True,) * dim)
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    p = np.array([0.3, -0.7, 1.1, 0.2])
    q = np.array([-0.4, 0.5, 0.0, 0.9])
    c = -0.6

    def f(x):
        row = np.floor(x[..., 1] * ny + 1e-9).astype(int) % ny
        comps = [p[row], np.full(x.shape[:-1], c)] + ([q[row]] if dim == 3 else [])
        return np.stack(comps, -1)

    x = sp.interpolate(f)
    area = 1.0 if dim == 2 else lengths[0] * lengths[2]
    jump2 = (p - np.roll(p, -1)) ** 2 + ((q - np.roll(q, -1)) ** 2 if dim == 3 else 0.0)
    D = 0.5 * abs(c) * area * np.sum(jump2)
    assert O.dissipation(sp, x, -1) == pytest.approx(D, rel=1e-12)
    r = O.residual(sp, x, -1)
    assert x @ r == pytest.approx(D, rel=1e-11)
    for l in range(0, k + 1):
        assert O.dissipation(sp, x, l) <= 1e-24
        assert abs(x @ O.residual(sp, x, l)) <= 1e-12 * D
    # jump indicator (end of section 3.2): |jump_j| / |<u>_j| on each facet
    # between rows j and j+1 (nx of them in 2D, 2 nx nz triangles in 3D), 0
    # on every other facet; 0 everywhere once Pi^l (l >= 0) removes the jump
    pn, qn = np.roll(p, -1), np.roll(q, -1)
    jmp = np.sqrt((p - pn) ** 2 + ((q - qn) ** 2 if dim == 3 else 0.0))
    avg = np.sqrt(((p + pn) / 2) ** 2 + c * c + (((q + qn) / 2) ** 2 if dim == 3 else 0.0))
    per_row = n[0] if dim == 2 else 2 * n[0] * n[2]
    want = np.concatenate([np.repeat(jmp / avg, per_row), np.zeros(sp.topo.n_facets - ny * per_row)])
    eta = O.jump_indicator(sp, x, -1)
    assert np.allclose(np.sort(eta), np.sort(want), rtol=1e-12, atol=1e-12)
    assert np.abs(O.jump_indicator(sp, x, 0)).max() <= 1e-12
    # kinetic energy 1/2 int |u|^2 and divergence of the piecewise-constant field
    vol_row = np.prod(lengths) / ny
    E = 0.5 * vol_row * np.sum(p ** 2 + c * c + (q ** 2 if dim == 3 else 0.0))
    assert O.energy(sp, x) == pytest.approx(E, rel=1e-13)
    assert O.divergence_l2(sp, x) <= 1e-13


def test_central_part_skew_symmetric_periodic(periodic2d):
    sp, f = periodic2d
    w = sp.interpolate(f, nq1d=10)
    A = O.assemble_picard(sp, w, -1, VOL | CEN)
    assert np.abs(A + A.T).max() <= 2e-12 * np.abs(A).max()


@pytest.mark.parametrize("which,nq", [("periodic2d", 10), ("periodic3d", 12)])
def test_energy_change_equals_dissipation(which, nq, request):
    """u^T r(u) = sum_E int 1/2 |u.n| |(I - Pi^l)[[u]]|^2 >= 0 on divergence-free u;
    zero for l = k (central)."""
    sp, f = request.getfixturevalue(which)
    x = sp.interpolate(f, nq1d=nq)
    x = x + 0.05 * divfree_random(sp, 3) if sp.n_dof < 3000 else x
    for l in (-1, 0, 1):
        r = O.residual(sp, x, l)
        D = O.dissipation(sp, x, l)
        assert D > 0
        assert abs(x @ r - D) <= 1e-11 * (abs(D) + minv_norm(sp, r) * m_norm(sp, x) * 1e-2)
    r = O.residual(sp, x, sp.k)
    assert abs(x @ r) <= 1e-12 * minv_norm(sp, r) * m_norm(sp, x)
    assert O.dissipation(sp, x, sp.k) <= 1e-20 * O.dissipation(sp, x, -1)


# ------------------------------------------------------------ brute force
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_brute_force_two_elements(dim, k):
    """Dense C(w) from double loops over physical basis products, applied to
    w, equals the matrix-free residual r(w) (arbitrary w, all l)."""
    m = two_element_mesh(dim)
    sp = S.Space(m.elem_vid, m.elem_xyz, k)
    w = np.random.default_rng(dim * 10 + k).standard_normal(sp.n_dof)
    # term scale: the standard-upwind matrix (the central one can vanish)
    scale = np.abs(O.assemble_picard(sp, w, -1)).max() * np.abs(w).max()
    for l in (-1, 0, k - 1, k):
        C = O.assemble_picard(sp, w, l)
        r = O.residual(sp, w, l)
        assert np.abs(C @ w - r).max() <= 1e-13 * scale


def test_brute_force_periodic(periodic2d):
    sp, f = periodic2d
    w = np.random.default_rng(4).standard_normal(sp.n_dof)
    C = O.assemble_picard(sp, w, 1)
    r = O.residual(sp, w, 1)
    assert np.abs(C @ w - r).max() <= 1e-13 * np.abs(C).max() * np.abs(w).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_standard_upwind_matches_eq_upwind(dim):
    """l = -1: the paper's eq. (upwind) in advective form equals the assembled
    conservative operator on divergence-free w."""
    m = two_element_mesh(dim)
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    w = divfree_random(sp, 11)
    C = O.assemble_picard(sp, w, -1)
    a = O.residual_advective(sp, w, -1)
    assert np.abs(C @ w - a).max() <= 1e-12 * np.abs(a).max()


# ------------------------------------------------------------ consistency
def test_convergence_taylor_green_2d():
    """M^{-1} r(Pi u) -> Pi (u.grad)u for 2D Taylor-Green,
    (u.grad)u = pi (sin 4 pi x, sin 4 pi y); observed order >= k - 0.2."""
    f = fields.taylor_green_2d()
    conv = lambda X: np.pi * np.stack([np.sin(4 * np.pi * X[..., 0]),
                                       np.sin(4 * np.pi * X[..., 1])], -1)
    for k in (1, 2, 3, 4):
        errs = []
        Ns = (8, 16, 32)
        for N in Ns:
            mm = kuhn_mesh(2, (N, N))
            sp = S.Space(mm.elem_vid, mm.elem_xyz, k)
            x = sp.interpolate(f, nq1d=k + 8)
            e = O.mass_solve(sp, O.residual(sp, x, k - 1)) - sp.interpolate(conv, nq1d=k + 8)
            errs.append(m_norm(sp, e))
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert rates[-1] >= k - 0.2, (k, errs, rates)


def test_convergence_taylor_green_3d():
    """M^{-1} r(Pi u) -> Pi (u.grad)u for 3D Taylor-Green on the periodic
    [0, 2 pi]^3, u = (sin x cos y cos z, -cos x sin y cos z, 0), where
    (u.grad)u = (1/2 sin 2x cos^2 z, 1/2 sin 2y cos^2 z, 0) in closed form;
    observed order >= k - 0.2 between the two finest meshes (k = 3 is still
    approaching its rate at N = 10: 2.67 from N = 4 to 8, 2.81 from 5 to 10,
    2.82 from 6 to 12).  The mass solves use the oracle's CG (the sparse LU
    of 10^5 3D unknowns takes minutes)."""
    f = fields.taylor_green_3d()
    conv = lambda X: np.stack([0.5 * np.sin(2 * X[..., 0]) * np.cos(X[..., 2]) ** 2,
                               0.5 * np.sin(2 * X[..., 1]) * np.cos(X[..., 2]) ** 2,
                               0.0 * X[..., 0]], -1)
    for k, Ns in ((1, (8, 16)), (2, (4, 8)), (3, (5, 10))):
        errs = []
        for N in Ns:
            mm = kuhn_mesh(3, (N, N, N), (2 * np.pi,) * 3)
            sp = S.Space(mm.elem_vid, mm.elem_xyz, k)
            x = sp.interpolate(f, nq1d=k + 5)
            e = O.mass_solve(sp, O.residual(sp, x, k - 1), method="cg") - sp.interpolate(conv, nq1d=k + 5)
            errs.append(m_norm(sp, e))
        rate = math.log2(errs[0] / errs[1])
        assert rate >= k - 0.2, (k, errs, rate)


# ------------------------------------------------------------ mass, substep
def test_mass_solve_and_l2_projection(wall3d):
    sp, _ = wall3d
    r = np.random.default_rng(1).standard_normal(sp.n_dof)
    w = O.mass_solve(sp, r)
    assert np.linalg.norm(O.mass_apply(sp, w) - r) <= 1e-13 * np.linalg.norm(r)
    # L2 projection of a field in V_h is the field itself
    f = fields.shear_field([0.2, 1.0, -0.8], [0.1, -0.5, 0.3])
    t = sp.topo
    b = np.zeros(sp.n_dof)
    for eb in sp.batches(t.n_elems, 64):
        phi = sp.phys_vals(eb, sp.ref_vals)
        u = f(sp.physical_points(eb, sp.xq))
        wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
        sp.scatter(b, eb, np.einsum("bq,bqd,bqid->bi", wdx, u, phi))
    x = sp.interpolate(f)
    assert np.abs(O.mass_solve(sp, b) - x).max() <= 1e-12 * np.abs(x).max()


def test_substep_energy_identity(periodic3d):
    """E(u - dt w) - E(u) = -dt u^T r + dt^2/2 r^T w with M w = r."""
    sp, f = periodic3d
    x = sp.interpolate(f, nq1d=10) + 1e-3 * np.random.default_rng(0).standard_normal(sp.n_dof)
    dt = 1e-2
    r = O.residual(sp, x, 1)
    w = O.mass_solve(sp, r)
    x1 = O.substep(sp, x, dt, 1)
    lhs = O.energy(sp, x1) - O.energy(sp, x)
    rhs = -dt * (x @ r) + 0.5 * dt * dt * (r @ w)
    assert abs(lhs - rhs) <= 1e-13 * O.energy(sp, x)


# ------------------------------------------------------------ adjoints
@pytest.mark.parametrize("which", ["periodic2d", "wall3d"])
def test_vjp_dot_product_and_homogeneity(which, request):
    sp, f = request.getfixturevalue(which)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(sp.n_dof)
    mu = rng.standard_normal(sp.n_dof)
    l = 1
    g = O.vjp(sp, x, mu, l)
    # r is positively homogeneous of degree 2: J_r(u) u = 2 r(u)
    assert abs(g @ x - 2 * (mu @ O.residual(sp, x, l))) <= 1e-12 * abs(g @ x) + 1e-12
    h = 1e-6
    for _ in range(3):
        dlt = rng.standard_normal(sp.n_dof)
        fd = mu @ (O.residual(sp, x + h * dlt, l) - O.residual(sp, x - h * dlt, l)) / (2 * h)
        assert abs(fd - g @ dlt) <= 1e-7 * abs(fd)


def test_chain_adjoint_fd():
    m, f, c = synth.make_config(1, n_override=(4, 4))
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    x0 = sp.interpolate(f, nq1d=10) + 1e-2 * np.random.default_rng(0).standard_normal(sp.n_dof)
    dt, n, l = 2e-2, 4, 1

    def loss(x):
        xN = O.substeps(sp, x, dt, n, l)
        return 0.5 * xN @ O.mass_apply(sp, xN)
    xN = O.substeps(sp, x0, dt, n, l)
    lam0 = O.chain_vjp(sp, x0, dt, n, l, O.mass_apply(sp, xN))
    rng = np.random.default_rng(9)
    h = 1e-6
    for _ in range(3):
        dlt = rng.standard_normal(sp.n_dof)
        dlt *= m_norm(sp, x0) / m_norm(sp, dlt)
        fd = (loss(x0 + h * dlt) - loss(x0 - h * dlt)) / (2 * h)
        assert abs(fd - lam0 @ dlt) <= 1e-7 * abs(fd)


# ------------------------------------------------------ adaptive order (NEXT f1)
def test_jump_indicator_properties(periodic2d):
    """eta vanishes for fields without jumps, is scale invariant, and with
    l = k the projected jump is zero."""
    sp, f = periodic2d
    c = sp.interpolate(fields.constant_field([0.4, -0.2]))
    assert np.abs(O.jump_indicator(sp, c, -1)).max() < 1e-12
    x = sp.interpolate(f, nq1d=10) + 1e-2 * np.random.default_rng(3).standard_normal(sp.n_dof)
    e1 = O.jump_indicator(sp, x, -1)
    assert np.allclose(O.jump_indicator(sp, 3.7 * x, -1), e1, rtol=1e-13)
    assert np.abs(O.jump_indicator(sp, x, sp.k)).max() < 1e-12 * e1.max()


def test_adapt_order_intervals():
    """The threshold rule of section 3.2 with the k = 3 thresholds of
    section 4 {0.1, 0.2, 0.3, 0.4}: eta_i < eta <= eta_{i+1} -> i, below
    eta_0 -> -1 (the hand-worked cases in tests/golden/adaptive_order_k3.txt)."""
    th, eta, want = None, [], []
    path = os.path.join(os.path.dirname(__file__), "golden", "adaptive_order_k3.txt")
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "thresholds":
            th = [float(v) for v in f[1:]]
        else:
            eta.append(float(f[0]))
            want.append(int(f[1]))
    assert th == [0.1, 0.2, 0.3, 0.4] and len(eta) >= 10
    assert np.array_equal(O.adapt_order(np.array(eta), th, 3), np.array(want))
