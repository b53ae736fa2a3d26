"""Reference-element polynomial spaces, facet polynomials, degrees of freedom
and the dual (nodal) basis of the velocity space (oracle; test infrastructure
only).

Velocity space (section 2.2, eq. (disc_velspace); reading: full vector P^k per
simplex with continuous normal component, i.e. BDM_k).  Its basis is the dual
basis of the following functionals, written on the reference simplex T^ with
vertices v0 = 0, vi = e_i:

  facet functionals, local facet i = facet opposite vertex i, with its other
  vertices a < b (< c) parametrised as x(s) = v_a + s1 (v_b - v_a)
  (+ s2 (v_c - v_a)), s in the reference (d-1)-simplex S^:
      N_i(v) = int_S^ (v(x(s)) . N^_i) psi_j(s) ds,
      N^_i = (v_b - v_a) x (v_c - v_a)       (3D)
      N^_i = R (v_b - v_a), R(t) = (t2, -t1)  (2D)
  psi_j: orthonormal polynomials on S^ (Legendre in 2D; the collapsed
  Dubiner family in 3D, ordered by total degree, then by the second index);

  interior functionals  I_m(v) = int_T^ v . q_m dx with, for x~ = x - barycentre,
      q = grad(x~^beta), 1 <= |beta| <= k-1 (graded lex: degree up, x1 > x2 > x3)
      then 2D: (-x~2, x~1) x~^beta, |beta| <= k-2
           3D: x~ x (e_i x~^beta), i = 1..3 outer, |beta| <= k-2 inner,
               skipping i = 1 with beta_1 >= 1.

The oracle represents P^k internally by the orthonormal Dubiner family
(collapsed Jacobi products, evaluated with scipy's Jacobi polynomials); the
internal basis does not change any result.
"""
import itertools
from functools import lru_cache
import numpy as np
from scipy.linalg import solve_triangular
from scipy.special import eval_jacobi, eval_legendre

from .quadrature import simplex_rule


# ---------------------------------------------------------------- multi-indices
def multi_indices(dim, kmax, kmin=0):
    """All exponent tuples with kmin <= |beta| <= kmax, graded lex order
    (degree ascending, then descending lexicographic: x1 > x2 > x3)."""
    out = []
    for deg in range(kmin, kmax + 1):
        level = [b for b in itertools.product(range(deg + 1), repeat=dim)
                 if sum(b) == deg]
        level.sort(reverse=True)
        out.extend(level)
    return out


def dim_P(dim, k):
    if k < 0:
        return 0
    if dim == 1:
        return k + 1
    if dim == 2:
        return (k + 1) * (k + 2) // 2
    return (k + 1) * (k + 2) * (k + 3) // 6


# ------------------------------------------------------- scalar P^k on T^
def _jac(n, a, x):
    return eval_jacobi(n, a, 0.0, x) if n >= 0 else np.zeros_like(x)


def _djac(n, a, x):
    """d/dx P_n^(a,0)(x) = (n + a + 1)/2 P_{n-1}^(a+1,1)(x)."""
    if n == 0:
        return np.zeros_like(x)
    return 0.5 * (n + a + 1) * eval_jacobi(n - 1, a + 1.0, 1.0, x)


def _collapsed_factor(i, a, x, t):
    """A(x, t) = t^i P_i^(a,0)(2x/t - 1) and its partial derivatives in x and t
    (polynomial in x and t; written with t^(i-1) so it stays finite)."""
    eta = 2.0 * x / t - 1.0
    P = _jac(i, a, eta)
    dP = _djac(i, a, eta)
    A = t ** i * P
    if i == 0:
        return A, np.zeros_like(x), np.zeros_like(x)
    Ax = t ** (i - 1) * 2.0 * dP
    At = t ** (i - 1) * (i * P - (1.0 + eta) * dP)
    return A, Ax, At


def scalar_modes(dim, k):
    if dim == 2:
        return [(i, j) for i in range(k + 1) for j in range(k + 1 - i)]
    return [(i, j, l) for i in range(k + 1) for j in range(k + 1 - i)
            for l in range(k + 1 - i - j)]


def scalar_basis(dim, k, x):
    """Orthonormal (Dubiner) basis of P^k(T^) at points x [N][dim]:
    values [N][nP], gradients [N][nP][dim].
      2D: p_ij  = c P_i(e1) ((1-e2)/2)^i P_j^(2i+1,0)(e2)
      3D: p_ijl = c P_i(e1) ((1-e2)/2)^i P_j^(2i+1,0)(e2) ((1-e3)/2)^(i+j)
                  P_l^(2i+2j+2,0)(e3)
    in collapsed coordinates, evaluated as products of polynomial factors in
    x1, t = 1 - x2 (- x3), s = 1 - x3."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    modes = scalar_modes(dim, k)
    vals = np.empty((x.shape[0], len(modes)))
    grads = np.empty((x.shape[0], len(modes), dim))
    if dim == 2:
        x1, x2 = x[:, 0], x[:, 1]
        t = 1.0 - x2
        for m, (i, j) in enumerate(modes):
            c = np.sqrt(2.0 * (2 * i + 1) * (i + j + 1))
            A, Ax, At = _collapsed_factor(i, 0.0, x1, t)
            Bv = _jac(j, 2 * i + 1.0, 2.0 * x2 - 1.0)
            dB = 2.0 * _djac(j, 2 * i + 1.0, 2.0 * x2 - 1.0)
            vals[:, m] = c * A * Bv
            grads[:, m, 0] = c * Ax * Bv
            grads[:, m, 1] = c * (-At * Bv + A * dB)
        return vals, grads
    x1, x2, x3 = x[:, 0], x[:, 1], x[:, 2]
    t = 1.0 - x2 - x3
    s = 1.0 - x3
    for m, (i, j, l) in enumerate(modes):
        c = np.sqrt((2 * i + 1.0) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * l + 3))
        A, Ax, At = _collapsed_factor(i, 0.0, x1, t)
        Bv, Bx, Bs = _collapsed_factor(j, 2 * i + 1.0, x2, s)
        a3 = 2 * i + 2 * j + 2.0
        Cv = _jac(l, a3, 2.0 * x3 - 1.0)
        dC = 2.0 * _djac(l, a3, 2.0 * x3 - 1.0)
        vals[:, m] = c * A * Bv * Cv
        grads[:, m, 0] = c * Ax * Bv * Cv
        grads[:, m, 1] = c * (-At * Bv * Cv + A * Bx * Cv)
        grads[:, m, 2] = c * (-At * Bv * Cv - A * Bs * Cv + A * Bv * dC)
    return vals, grads


# ------------------------------------------------------------ facet psi_j
def facet_modes(dim, k):
    """Ordered list of facet mode labels: 2D: j; 3D: (p, q) ordered by
    m = p + q ascending, then q ascending."""
    if dim == 2:
        return [(j,) for j in range(k + 1)]
    out = []
    for m in range(k + 1):
        for q in range(m + 1):
            out.append((m - q, q))
    return out


def facet_mode_degree(mode):
    return sum(mode)


def psi(dim, k, s):
    """Orthonormal facet polynomials psi_j(s) on S^ (param measure),
    s: [N][dim-1] -> [N][n_f].
      2D: psi_j = sqrt(2j+1) P_j(2s-1)
      3D: psi_pq = sqrt(2(2p+1)(p+q+1)) P_p(e1) ((1-e2)/2)^p P_q^(2p+1,0)(e2),
          e1 = 2 s1/(1 - s2) - 1, e2 = 2 s2 - 1."""
    s = np.atleast_2d(s)
    modes = facet_modes(dim, k)
    out = np.empty((s.shape[0], len(modes)))
    if dim == 2:
        for j, (jj,) in enumerate(modes):
            out[:, j] = np.sqrt(2 * jj + 1.0) * eval_legendre(jj, 2.0 * s[:, 0] - 1.0)
        return out
    s1, s2 = s[:, 0], s[:, 1]
    e2 = 2.0 * s2 - 1.0
    e1 = 2.0 * s1 / (1.0 - s2) - 1.0
    for j, (p, q) in enumerate(modes):
        c = np.sqrt(2.0 * (2 * p + 1) * (p + q + 1))
        out[:, j] = (c * eval_legendre(p, e1) * ((1.0 - e2) / 2.0) ** p
                     * eval_jacobi(q, 2 * p + 1.0, 0.0, e2))
    return out


# ---------------------------------------------------- reference facets
def ref_vertices(dim):
    return np.vstack([np.zeros(dim), np.eye(dim)])


def facet_local_vertices(dim, i):
    """Local vertex indices of local facet i (opposite vertex i), ascending."""
    return [v for v in range(dim + 1) if v != i]


def rotate_2d(t):
    return np.array([t[1], -t[0]])


def ref_facet_map(dim, i):
    """(origin, edge matrix [dim][dim-1], unnormalised normal N^_i) such that
    x(s) = origin + E s."""
    V = ref_vertices(dim)
    lv = facet_local_vertices(dim, i)
    o = V[lv[0]]
    E = np.stack([V[v] - o for v in lv[1:]], 1)
    if dim == 2:
        N = rotate_2d(E[:, 0])
    else:
        N = np.cross(E[:, 0], E[:, 1])
    return o, E, N


# ---------------------------------------------------- interior test fields
def interior_tests(dim, k, x):
    """q_m at points x [N][dim] -> [N][n_int][dim] (see module docstring)."""
    x = np.atleast_2d(x)
    xt = x - 1.0 / (dim + 1)
    fields = []
    for beta in multi_indices(dim, k - 1, 1):
        g = np.zeros((x.shape[0], dim))
        for a in range(dim):
            if beta[a] == 0:
                continue
            e = list(beta)
            e[a] -= 1
            g[:, a] = beta[a] * np.prod(xt ** np.array(e), axis=1)
        fields.append(g)
    for_betas = multi_indices(dim, k - 2, 0) if k >= 2 else []
    if dim == 2:
        for beta in for_betas:
            m = np.prod(xt ** np.array(beta), axis=1)
            fields.append(np.stack([-xt[:, 1] * m, xt[:, 0] * m], -1))
    else:
        for i in range(3):
            for beta in for_betas:
                if i == 0 and beta[0] >= 1:
                    continue
                m = np.prod(xt ** np.array(beta), axis=1)
                e = np.zeros((x.shape[0], 3))
                e[:, i] = m
                fields.append(np.cross(xt, e))
    if not fields:
        return np.zeros((x.shape[0], 0, dim))
    return np.stack(fields, 1)


def n_facet_dofs(dim, k):
    return dim_P(dim - 1, k)


def n_interior_dofs(dim, k):
    return dim * dim_P(dim, k) - (dim + 1) * n_facet_dofs(dim, k)


# ---------------------------------------------------- DoF matrix, dual basis
@lru_cache(maxsize=None)
def dof_matrix(dim, k):
    """D^[i, (a, alpha)] = functional_i(e_a p_alpha), n x n, with the local
    DoF order: facets 0..d (facet modes inner), then interior functionals.
    Vector modal index (a, alpha) -> a * nP + alpha."""
    nP = dim_P(dim, k)
    nf = n_facet_dofs(dim, k)
    n = dim * nP
    D = np.zeros((n, n))
    # facet functionals
    s, ws = simplex_rule(dim - 1, k + 2)
    ps = psi(dim, k, s)  # [ns][nf]
    for i in range(dim + 1):
        o, E, N = ref_facet_map(dim, i)
        xh = o[None, :] + s @ E.T
        pv, _ = scalar_basis(dim, k, xh)  # [ns][nP]
        for a in range(dim):
            # int (p_alpha N_a) psi_j ds
            blk = (ps * ws[:, None]).T @ (pv * N[a])  # [nf][nP]
            D[i * nf:(i + 1) * nf, a * nP:(a + 1) * nP] = blk
    # interior functionals
    x, w = simplex_rule(dim, k + 2)
    pv, _ = scalar_basis(dim, k, x)
    q = interior_tests(dim, k, x)  # [N][nint][dim]
    r0 = (dim + 1) * nf
    for a in range(dim):
        D[r0:, a * nP:(a + 1) * nP] = (q[:, :, a] * w[:, None]).T @ pv
    return D


@lru_cache(maxsize=None)
def dual_coefficients(dim, k):
    """C = D^{-1}: reference dual basis phi^_i = sum C[(a,alpha), i] e_a p_alpha."""
    return np.linalg.inv(dof_matrix(dim, k))


def dual_basis(dim, k, x):
    """Reference dual basis at points x [N][dim]:
    values [N][n][dim], gradients [N][n][dim(component)][dim(derivative)]."""
    nP = dim_P(dim, k)
    C = dual_coefficients(dim, k)
    pv, pg = scalar_basis(dim, k, x)
    n = dim * nP
    vals = np.empty((pv.shape[0], n, dim))
    grads = np.empty((pv.shape[0], n, dim, dim))
    for a in range(dim):
        Ca = C[a * nP:(a + 1) * nP, :]  # [nP][n]
        vals[:, :, a] = pv @ Ca
        grads[:, :, a, :] = np.einsum("qpb,pi->qib", pg, Ca)
    return vals, grads
