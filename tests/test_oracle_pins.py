"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Each test names the property and where it comes from.  None of them re-types
the oracle's own formula: they check closed forms, invariants, special cases
and brute-force evaluations on tiny inputs.
"""
import math
import itertools
import numpy as np
import pytest

import synth
from oracle import basis as B, quadrature as Q, mesh as OM, space as S, operator as O
from synth.mesh import kuhn_mesh, two_element_mesh


# ------------------------------------------------------------- quadrature
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_quadrature_monomials_closed_form(dim, n):
    """int_T^ x^beta = beta! / (|beta| + d)! (Dirichlet integral), exact up to
    total degree 2n - 1 for the collapsed Gauss-Jacobi rule."""
    x, w = Q.simplex_rule(dim, n)
    assert abs(w.sum() - 1.0 / math.factorial(dim)) < 1e-15
    for deg in range(2 * n):
        for beta in itertools.product(range(deg + 1), repeat=dim):
            if sum(beta) != deg:
                continue
            exact = np.prod([math.factorial(b) for b in beta]) / math.factorial(deg + dim)
            val = np.sum(w * np.prod(x ** np.array(beta), axis=1))
            assert abs(val - exact) <= 1e-14 * max(exact, 1e-300) + 1e-17


def test_quadrature_degree_choice():
    """Volume rule integrates degree 3k-1, facet rule degree 3k."""
    for k in range(1, 7):
        assert 2 * Q.volume_points_per_dir(k) - 1 >= 3 * k - 1
        assert 2 * Q.facet_points_per_dir(k) - 1 >= 3 * k


# ------------------------------------------------------------- bases
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_scalar_basis_orthonormal(dim, k):
    x, w = Q.simplex_rule(dim, k + 1)
    v, _ = B.scalar_basis(dim, k, x)
    G = (v * w[:, None]).T @ v
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_scalar_gradients_divergence_theorem(dim, k):
    """int_T^ d_b p = int_{dT^} p n_b ds for every basis function (exact
    rules on both sides): pins the gradients independently of the values."""
    x, w = Q.simplex_rule(dim, k + 1)
    _, g = B.scalar_basis(dim, k, x)
    lhs = np.einsum("q,qpb->pb", w, g)
    rhs = np.zeros_like(lhs)
    s, ws = Q.simplex_rule(dim - 1, k + 1)
    for i in range(dim + 1):
        o, E, N = B.ref_facet_map(dim, i)
        sign = (-1.0) ** i  # outward orientation of N^_i on the reference simplex
        v, _ = B.scalar_basis(dim, k, o[None, :] + s @ E.T)
        # ds_phys = |N^| ds_param and n = sign N^/|N^|
        rhs += np.einsum("q,qp,b->pb", ws, v, sign * N)
    assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_facet_psi_orthonormal_and_counts(dim, k):
    s, w = Q.simplex_rule(dim - 1, k + 1)
    p = B.psi(dim, k, s)
    assert p.shape[1] == B.dim_P(dim - 1, k)
    G = (p * w[:, None]).T @ p
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13
    # degrees ascending
    degs = [B.facet_mode_degree(m) for m in B.facet_modes(dim, k)]
    assert degs == sorted(degs)


def test_dof_counts():
    """n_int = d dim P^k - (d+1) dim P^k(facet): 3, 20, 45, 84 for the
    workloads (2D k=2; 3D k=3,4,5), and 168 local DoFs at 3D k=5."""
    assert B.n_interior_dofs(2, 2) == 3
    assert [B.n_interior_dofs(3, k) for k in (3, 4, 5)] == [20, 45, 84]
    assert 3 * B.dim_P(3, 5) == 168
    for dim in (2, 3):
        for k in range(1, 7):
            q = B.interior_tests(dim, k, np.zeros((1, dim)) + 0.2)
            assert q.shape[1] == B.n_interior_dofs(dim, k)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_dual_basis_identity(dim, k):
    D = B.dof_matrix(dim, k)
    C = B.dual_coefficients(dim, k)
    # relative to row scale (the interior functionals have small norms)
    R = D @ C - np.eye(D.shape[0])
    assert np.abs(R).max() < 1e-10
    assert np.abs(C @ D - np.eye(D.shape[0])).max() < 1e-9


def _element_functionals(sp, e, values_at_facet, values_at_vol, rule_n):
    """Apply the physical DoF functionals of element e to a field given as
    callables of reference points (facet i, s) and (x^)."""
    t = sp.topo
    d = sp.dim
    out = []
    s, ws = Q.simplex_rule(d - 1, rule_n)
    ps = B.psi(d, sp.k, s)
    for i in range(d + 1):
        lv = [v for v in range(d + 1) if v != i]
        xv = t.xyz[e, lv]
        # physical normal straight from the physical vertices
        N = OM.facet_vectors(xv[None], d)[0]
        n = N / np.linalg.norm(N)
        u = values_at_facet(i, s)  # [ns][d] physical field
        out.append(((u @ n) * ws) @ ps)
    x, w = Q.simplex_rule(d, rule_n)
    u = values_at_vol(x)
    J = t.J[e]
    uh = (t.detJ[e] * np.linalg.solve(J, u.T)).T
    q = B.interior_tests(d, sp.k, x)
    out.append(np.abs(t.detJ[e]) ** (-(d - 1) / d) * np.einsum("qj,qmj,q->m", uh, q, w))
    return np.concatenate(out)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_delta_property_random_elements(dim, k):
    """DoF_i(phi_{T,j}) = delta_ij for the physical basis on random affine
    elements, including ones with det J < 0."""
    rng = np.random.default_rng(12 + dim + k)
    m = two_element_mesh(dim)
    sp = S.Space(m.elem_vid, m.elem_xyz, k)
    for trial in range(3):
        xyz = rng.standard_normal((1, dim + 1, dim))
        vid = np.arange(dim + 1)[None, :]
        t = OM.build(vid, xyz)
        sp.topo = t  # a one-element view for the physical basis helpers
        sp.S = np.empty((1, sp.n))
        for i in range(dim + 1):
            sp.S[0, i * sp.nf:(i + 1) * sp.nf] = t.NF_norm[0, i]
        sp.S[0, (dim + 1) * sp.nf:] = abs(t.detJ[0]) ** ((dim - 1) / dim)
        sp.Jinv = np.linalg.inv(t.J)
        M = np.empty((sp.n, sp.n))
        for j in range(sp.n):
            def vf(i, s, j=j):
                o, E, _ = B.ref_facet_map(dim, i)
                vals, _ = B.dual_basis(dim, k, o[None, :] + s @ E.T)
                return sp.phys_vals(np.array([0]), vals)[0, :, j, :]

            def vv(x, j=j):
                vals, _ = B.dual_basis(dim, k, x)
                return sp.phys_vals(np.array([0]), vals)[0, :, j, :]
            M[:, j] = _element_functionals(sp, 0, vf, vv, k + 2)
        assert np.abs(M - np.eye(sp.n)).max() < 1e-10, (trial, t.detJ)


# ------------------------------------------------------------- mesh
@pytest.mark.parametrize("cfg", [1, 3])
def test_geometry_invariants(cfg):
    n = (6, 6) if cfg == 1 else (4, 5, 4)
    m, f, c = synth.make_config(cfg, n_override=n)
    t = OM.build(m.elem_vid, m.elem_xyz)
    vol = np.sum(np.abs(t.detJ)) / math.factorial(t.dim)
    assert abs(vol - np.prod(c["lengths"])) < 1e-13
    # closed surfaces: sum_i sigma_i N_{F_i} = 0
    closure = np.einsum("ei,eid->ed", t.sigma, t.NF)
    assert np.abs(closure).max() < 1e-14 * np.abs(t.NF).max() * 10
    for e in range(t.n_elems):
        for i in range(t.dim + 1):
            nb = t.nbr[e, i]
            if nb >= 0:
                assert t.nbr[nb, t.nbr_face[e, i]] == e
                # the same facet normal from both sides
                assert np.allclose(t.NF[e, i], t.NF[nb, t.nbr_face[e, i]], atol=1e-14)
    # facet points coincide modulo the period
    L = np.array(c["lengths"])
    for f_ in range(0, t.n_facets, 7):
        (e0, e1), (i0, i1) = t.facet_elems[f_], t.facet_local[f_]
        p0 = t.xyz[e0, [v for v in range(t.dim + 1) if v != i0]]
        p1 = t.xyz[e1, [v for v in range(t.dim + 1) if v != i1]]
        dlt = (p0 - p1) / L
        assert np.abs(dlt - np.round(dlt)).max() < 1e-12


def test_mesh_errors():
    with pytest.raises(ValueError):
        kuhn_mesh(2, (2, 4))
    vid = np.array([[0, 1, 2], [0, 1, 2], [0, 1, 2]])
    xyz = np.random.default_rng(0).standard_normal((3, 3, 2))
    with pytest.raises(OM.MeshError):
        OM.build(vid, xyz)
    with pytest.raises(OM.MeshError):
        OM.build(np.array([[0, 0, 1]]), xyz[:1])


# ------------------------------------------------------------- space
def _poly_field(dim, k, seed):
    rng = np.random.default_rng(seed)
    idx = B.multi_indices(dim, k)
    coef = rng.standard_normal((len(idx), dim))

    def f(x):
        out = np.zeros(x.shape)
        for c, beta in zip(coef, idx):
            out += np.prod(x ** np.array(beta), axis=-1)[..., None] * c
        return out
    return f


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 2), (3, 3)])
def test_interpolation_reproduces_polynomials(dim, k):
    m = kuhn_mesh(dim, (3,) * dim, periodic=(False,) * dim, jitter=0.1, jitter_seed=5)
    # a wall mesh would force u.n = 0; use a mesh where every facet is interior
    # by sampling on a periodic mesh with a periodic polynomial-free check below
    sp = S.Space(m.elem_vid, m.elem_xyz, k)
    # polynomial fields are only in V_h if their normal trace vanishes on walls;
    # test the element-local identity instead: evaluate the interpolant at
    # interior points of elements touching no wall facet
    f = _poly_field(dim, k, 3)
    x = sp.interpolate(f)
    inner = np.nonzero(np.all(sp.topo.elem_facet >= 0, axis=1))[0]
    assert len(inner) > 0
    pts = np.random.default_rng(1).uniform(0, 1.0 / (dim + 1), (7, dim))
    val = sp.evaluate(x, inner, pts)
    ref = f(sp.physical_points(inner, pts))
    assert np.abs(val - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("cfg,n,k,nq", [(1, (8, 8), 2, 10), (1, (6, 6), 3, 11),
                                       (4, (4, 4, 4), 3, 14)])
def test_interpolant_commutes_with_div(cfg, n, k, nq):
    """div V_h subset Q_h (eq. (divVeqQ)) and the commuting interpolant keep a
    divergence-free field divergence-free to round-off when the DoF integrals of the analytic
    field are computed accurately (enough points per direction)."""
    m, f, c = synth.make_config(cfg, n_override=n)
    sp = S.Space(m.elem_vid, m.elem_xyz, k)
    x = sp.interpolate(f, nq1d=nq)
    assert O.divergence_l2(sp, x) <= 1e-12 * math.sqrt(2 * O.energy(sp, x))


def test_normal_continuity_random_coefficients():
    """u^T . n = u^T' . n at every facet point for arbitrary coefficients."""
    m, f, c = synth.make_config(3, n_override=(3, 4, 3))
    sp = S.Space(m.elem_vid, m.elem_xyz, 2)
    x = np.random.default_rng(2).standard_normal(sp.n_dof)
    fb = np.arange(sp.topo.n_facets)
    T, T2, phiT, phiT2, nvec, ds = O._facet_traces(sp, fb)
    uT = np.einsum("bqid,bi->bqd", phiT, sp.local(x, T))
    uT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(x, T2))
    jn = np.einsum("bqd,bd->bq", uT - uT2, nvec)
    assert np.abs(jn).max() < 1e-12 * np.abs(uT).max()
    # and equals sum_j x_{F,j} psi_j
    un = np.einsum("bqd,bd->bq", uT, sp.topo.NF[T, sp.topo.facet_local[:, 0]]
                   / sp.topo.NF_norm[T, sp.topo.facet_local[:, 0]][:, None])
    xf = x[:sp.topo.n_facets * sp.nf].reshape(-1, sp.nf)
    assert np.abs(un - xf @ sp.psi_q.T).max() < 1e-12 * np.abs(un).max()


# ------------------------------------------------------------ diagnostics
def walled_parabola_case(dim, k, jitter=0.05):
    """u = (0, y(1 - y)) in 2D, (0, y(1 - y), 0) in 3D, on a box of lengths
    (1.3, 1) or (1.5, 1, 0.5), periodic in x (and z), with walls at y = 0, 1,
    graded in y and jittered.  u is a polynomial of degree 2 with u.n = 0 on
    the walls, so it lies in V_h for k >= 2 and the canonical interpolant
    reproduces it; div u = 1 - 2y, so ||div u||^2 = (box area across y) / 3."""
    from synth.mesh import graded_nodes
    n = (3, 4) if dim == 2 else (3, 4, 3)
    lengths = (1.3, 1.0) if dim == 2 else (1.5, 1.0, 0.5)
    periodic = (True, False) if dim == 2 else (True, False, True)
    y = graded_nodes(n[1], 1.4, 1.0)
    nodes = [None] * dim
    nodes[1] = y / y[-1]
    mesh = kuhn_mesh(dim, n, lengths, periodic, nodes, jitter=jitter, jitter_seed=17)
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)

    def f(x):
        yy = x[..., 1]
        comps = [0.0 * yy, yy * (1.0 - yy)] + ([0.0 * yy] if dim == 3 else [])
        return np.stack(comps, -1)

    area = lengths[0] * (lengths[2] if dim == 3 else 1.0)
    return sp, sp.interpolate(f), math.sqrt(area / 3.0), mesh


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_divergence_l2_closed_form(dim, k):
    """||div u_h||_L2 (the substep diagnostic, with div u|_T = div^ u^/det J)
    equals the closed form for a parabola in V_h on a graded, jittered,
    walled mesh; the same field scaled by 3 gives 3 times the value."""
    sp, x, want, _ = walled_parabola_case(dim, k)
    assert O.divergence_l2(sp, x) == pytest.approx(want, rel=1e-13)
    assert O.divergence_l2(sp, 3.0 * x) == pytest.approx(3.0 * want, rel=1e-13)


def test_interpolation_restricted_to_elements():
    """Space.interpolate(..., elems=E') gives the full interpolant's DoFs on
    the elements E' (their facets and interiors) and zero elsewhere (the
    full-size tests use it to build inputs on a patch)."""
    m, f, c = synth.make_config(3, n_override=(3, 4, 3))
    sp = S.Space(m.elem_vid, m.elem_xyz, 3)
    x = sp.interpolate(f, nq1d=5)
    el = np.array([3, 17, 40, 41])
    xr = sp.interpolate(f, nq1d=5, elems=el)
    g = np.unique(sp.gdof[el][sp.gdof[el] >= 0])
    assert np.abs(xr[g] - x[g]).max() <= 1e-14 * np.abs(x).max()
    rest = np.setdiff1d(np.arange(sp.n_dof), g)
    assert not xr[rest].any()
