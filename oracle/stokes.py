"""Implicit Stokes step of the operator splitting (oracle; test
infrastructure only).

Paper section 2.2 (spaces Sigma_h, W_h, V^_h; forms a_h, b_2h) and section
2.3 (eq. (MCS_step1), its matrix form, the static condensation of sigma and
gamma, and the element-wise BDDC preconditioner without primal constraints).

Given u^n in V_h, nu and dt, find (sigma, u*, u^, gamma) in
Sigma_h x V_h x V^_h x W_h with

  a(sigma, tau) + b2(tau, (u*, u^, gamma)) = 0                    all tau
  (u* - u^n, v)/dt + b2(sigma, (v, v^, eta)) + c(u^n, u^n, v) = 0  all (v, v^, eta)

  a(sigma, tau)  = -1/(2 nu) sum_T int_T sigma : tau
  b2(sigma, (v, v^, eta)) = sum_T [ -int_T (div sigma) . v + int_dT sigma_nn (v . n)
                                   - int_T sigma : eta + int_dT sigma_nt . v^ ]

The convection term c(u^n, u^n, v) enters as a given vector r (the residual
of the convection operator at u^n, oracle.operator.residual); r = None
leaves it out (the Stokes part alone).

Readings (the paper does not fix them):
  * div of a matrix field is taken row by row, (div tau)_i = sum_j d_j tau_ij,
    so that int_T (div tau) . v = -int_T tau : grad v + int_dT (tau n) . v;
    tau_nn = n . tau n and tau_nt = tau n - tau_nn n (the tangential part of
    tau n);
  * Sigma_h: trace-free P^{k+1} matrices per element whose nt-trace has
    degree <= k on every interior facet (F^I, the paper's definition); on
    wall facets the nt-trace keeps degree k + 1;
  * W_h: skew-symmetric P^k matrices per element;
  * V^_h: on each interior facet F, tangential P^k vector fields
    u^ = sum_c sum_j u^_{F,c,j} psi_j(s) t_{F,c}, with psi_j the orthonormal
    facet polynomials of the velocity DoFs (oracle.basis.psi) on the facet's
    sorted-vertex parametrisation and the unit tangents
      2D: t = (x_b - x_a)/|x_b - x_a|,
      3D: t_1 = (x_b - x_a)/|x_b - x_a|, t_2 = n_F x t_1,
    x_a < x_b the facet's first two vertices in sorted id order and n_F its
    unit normal (oracle.mesh).  u^ = 0 on wall facets (no-slip), so wall
    facets carry no u^ unknowns.  Global layout: facet, tangent, mode (mode
    fastest).
  * every form is integrated exactly (end of section 2.2): k + 2 points per
    collapsed direction in volumes and on facets.

Bases inside the oracle (they do not change u*, u^, gamma or the function
sigma): the full trace-free space is spanned by the unit matrices e_i e_j^T
(i != j) and e_i e_i^T - e_d e_d^T, times monomials (x^ - x^_c)^beta of the
element's reference coordinates x^ = F_T^-1(x) (x^_c the reference
barycentre; an affine map keeps polynomial degrees, so this spans P^{k+1}
of the element, and it stays well conditioned on flat elements, where
monomials of physical coordinates do not); Sigma_T is the null space
(scipy.linalg.null_space, a library primitive) of the facet constraints.
W_T uses the skew unit matrices times the same monomials up to degree k.

Functions:
  step1(sp, un, nu, dt, r=None)        the saddle-point system of eq.
                                       (MCS_step1) assembled and solved
                                       directly (sparse LU): the definition;
  schur_system(sp, nu, dt)             the condensed matrix S = A - B M^-1 B^t
                                       (section 2.3) and the element blocks S_T;
  step1_condensed(sp, un, nu, dt, r)   S [u*; u^] = [M u^n/dt - r; 0], direct;
  bddc_apply(sp, blocks, x)            C^-1 x = R S_BDDC^-1 R^t x;
  step1_pcg(...)                       PCG on S with C^-1 (the paper's solver).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sps
import scipy.sparse.linalg as spla
from threadpoolctl import threadpool_limits

from . import basis as B
from .quadrature import simplex_rule


# ----------------------------------------------------------- matrix bases
def tracefree_basis(d):
    """e_i e_j^T (i != j), then e_i e_i^T - e_d e_d^T (i < d)."""
    out = []
    for i in range(d):
        for j in range(d):
            if i != j:
                m = np.zeros((d, d))
                m[i, j] = 1.0
                out.append(m)
    for i in range(d - 1):
        m = np.zeros((d, d))
        m[i, i] = 1.0
        m[d - 1, d - 1] = -1.0
        out.append(m)
    return np.array(out)


def skew_basis(d):
    """e_i e_j^T - e_j e_i^T, i < j."""
    out = []
    for i in range(d):
        for j in range(i + 1, d):
            m = np.zeros((d, d))
            m[i, j] = 1.0
            m[j, i] = -1.0
            out.append(m)
    return np.array(out)


def _monomials(d, deg, y):
    """((x - x_c)/h)^beta for |beta| <= deg at scaled points y [N][d]:
    values [N][nm] and gradients in y [N][nm][d]."""
    betas = B.multi_indices(d, deg)
    y = np.atleast_2d(y)
    vals = np.empty((y.shape[0], len(betas)))
    grads = np.zeros((y.shape[0], len(betas), d))
    for m, b in enumerate(betas):
        b = np.array(b)
        vals[:, m] = np.prod(y ** b, axis=1)
        for a in range(d):
            if b[a] == 0:
                continue
            e = b.copy()
            e[a] -= 1
            grads[:, m, a] = b[a] * np.prod(y ** e, axis=1)
    return vals, grads


# ----------------------------------------------------------- facet frames
def facet_frame(sp, T, i):
    """Unit normal n_F of the facet's sorted-vertex parametrisation, its
    tangents t_c [d-1][d], |N_F| and the outward sign for T."""
    t = sp.topo
    d = sp.dim
    lv = [v for v in range(d + 1) if v != i]
    xv = t.xyz[T, lv]
    nF = t.NF[T, i] / t.NF_norm[T, i]
    t1 = xv[1] - xv[0]
    t1 = t1 / np.linalg.norm(t1)
    if d == 2:
        tang = t1[None, :]
    else:
        tang = np.stack([t1, np.cross(nF, t1)])
    return nF, tang, t.NF_norm[T, i], t.sigma[T, i], xv


def n_uhat(sp):
    return sp.topo.n_facets * (sp.dim - 1) * sp.nf


def uhat_gdof(sp):
    """[E][(d+1)(d-1)n_f] global index of each element's local u^ unknown
    (facet, tangent, mode), -1 on wall facets."""
    t = sp.topo
    d, nf = sp.dim, sp.nf
    g = -np.ones((t.n_elems, (d + 1) * (d - 1) * nf), dtype=np.int64)
    for i in range(d + 1):
        f = t.elem_facet[:, i]
        for c in range(d - 1):
            for j in range(nf):
                col = (i * (d - 1) + c) * nf + j
                g[:, col] = np.where(f >= 0, (f * (d - 1) + c) * nf + j, -1)
    return g


# ----------------------------------------------------------- element blocks
def _ref_tabs(sp):
    """Reference dual-basis values at the Stokes rules (k + 2 points per
    direction), per space: volume [q][n][d] and each facet's [q][n][d]."""
    tab = getattr(sp, "_stokes_tabs", None)
    if tab is None:
        d, k = sp.dim, sp.k
        xq, wq = simplex_rule(d, k + 2)
        s, ws = simplex_rule(d - 1, k + 2)
        fac = []
        for i in range(d + 1):
            o, Em, _ = B.ref_facet_map(d, i)
            fac.append(B.dual_basis(d, k, o[None, :] + s @ Em.T)[0])
        tab = (xq, wq, B.dual_basis(d, k, xq)[0], s, ws, fac)
        sp._stokes_tabs = tab
    return tab


def element_blocks(sp, T, nu):
    """Blocks of eq. (MCS_step1)'s matrix form for element T, on the local
    Sigma_T basis: Mss [ns][ns], Bgs [ng][ns], Bus [n][ns], Bhs [nh][ns], the
    basis N (full trace-free monomial coefficients -> Sigma_T) and the
    reference barycentre of the monomials.  Full-space index of E_a mono_m:
    a * nm + m."""
    t = sp.topo
    d, k = sp.dim, sp.k
    Ea = tracefree_basis(d)
    Gc = skew_basis(d)
    J, detJ = t.J[T], t.detJ[T]
    x0 = t.xyz[T, 0]
    xc = np.full(d, 1.0 / (d + 1))            # reference barycentre
    Jinv = np.linalg.inv(J)
    xq_ref, wq_ref, ref_vals, s_ref, ws_ref, ref_face = _ref_tabs(sp)

    # volume terms in physical coordinates
    xq = x0[None, :] + xq_ref @ J.T
    wq = wq_ref * abs(detJ)
    mv, mg = _monomials(d, k + 1, xq_ref - xc)
    mg = mg @ Jinv                                # physical gradients: grad^ m J^-1
    gv, _ = _monomials(d, k, xq_ref - xc)
    phi = sp.phys_vals(np.array([T]), ref_vals)[0]  # [q][n][d]
    # a(sigma, tau) = -1/(2 nu) int sigma : tau
    Mfull = -np.kron(np.einsum("aij,bij->ab", Ea, Ea), (mv * wq[:, None]).T @ mv) / (2.0 * nu)
    # -int sigma : eta, eta = G_c mono_m'
    Bg_full = -np.kron(np.einsum("cij,aij->ca", Gc, Ea), (gv * wq[:, None]).T @ mv)
    # -int (div sigma) . v, (div E_a mono_m)_r = sum_s (E_a)_rs d_s mono_m
    Bu_full = np.concatenate([
        -sum(Ea[a, r, s_] * ((phi[:, :, r] * wq[:, None]).T @ mg[:, :, s_])
             for r in range(d) for s_ in range(d)) for a in range(len(Ea))], 1)

    # facet terms and the nt constraints
    nh_loc = (d + 1) * (d - 1) * sp.nf
    Bh_full = np.zeros((nh_loc, Bu_full.shape[1]))
    psi_k = B.psi(d, k, s_ref)                                    # [ns][nf]
    top = [m for m, mode in enumerate(B.facet_modes(d, k + 1))
           if B.facet_mode_degree(mode) == k + 1]
    psi_top = B.psi(d, k + 1, s_ref)[:, top]
    cons = []
    for i in range(d + 1):
        nF, tang, NFn, sgn, xv = facet_frame(sp, T, i)
        nout = sgn * nF
        ds = ws_ref * NFn
        o, Em, _ = B.ref_facet_map(d, i)
        fv, _ = _monomials(d, k + 1, o[None, :] + s_ref @ Em.T - xc)
        # v . n_out of the local velocity basis on this facet
        vn = sp.phys_vals(np.array([T]), ref_face[i])[0] @ nout   # [q][n]
        # sigma_nn of E_a mono_m is (n.E_a n) mono_m
        enn = np.einsum("i,aij,j->a", nout, Ea, nout)
        Bu_full += np.kron(enn[None, :], (vn * ds[:, None]).T @ fv)
        for c in range(d - 1):
            # (sigma n_out) . t_c and n_F . sigma t_c of E_a mono_m
            ent = np.einsum("i,aij,j->a", tang[c], Ea, nout)
            rows = (i * (d - 1) + c) * sp.nf + np.arange(sp.nf)
            Bh_full[rows] = np.kron(ent[None, :], (psi_k * ds[:, None]).T @ fv)
            if t.elem_facet[T, i] >= 0:
                etn = np.einsum("i,aij,j->a", nF, Ea, tang[c])
                cons.append(np.kron(etn[None, :], (psi_top * ws_ref[:, None]).T @ fv))
    if cons:
        C = np.concatenate(cons)
        N = sla.null_space(C, rcond=1e-12)
    else:
        N = np.eye(Bu_full.shape[1])
    return dict(N=N, Mss=N.T @ Mfull @ N, Bgs=Bg_full @ N, Bus=Bu_full @ N,
                Bhs=Bh_full @ N, xc=xc)


def expected_sigma_dim(d, k, n_interior_facets):
    """dim Sigma_T: trace-free P^{k+1} minus (d-1) (dim P^{k+1}(F) - dim P^k(F))
    constraints per interior facet."""
    top = B.dim_P(d - 1, k + 1) - B.dim_P(d - 1, k)
    return (d * d - 1) * B.dim_P(d, k + 1) - n_interior_facets * (d - 1) * top


def all_blocks(sp, nu):
    # small dense element matrices: one BLAS thread (many threads on
    # matrices this size only contend)
    with threadpool_limits(1):
        return [element_blocks(sp, T, nu) for T in range(sp.topo.n_elems)]


def _mass_local(sp, T):
    t = sp.topo
    phi = sp.phys_vals(np.array([T]), sp.ref_vals)[0]
    return np.einsum("q,qid,qjd->ij", sp.wq * abs(t.detJ[T]), phi, phi)


# ----------------------------------------------------------- direct solve
def step1(sp, un, nu, dt, r=None, blocks=None):
    """Solve eq. (MCS_step1) directly.  Returns (u*, u^, sigma [list of
    per-element coefficient vectors on Sigma_T], gamma [E][ng], blocks)."""
    from .operator import mass_matrix
    t = sp.topo
    E, d = t.n_elems, sp.dim
    blocks = blocks or all_blocks(sp, nu)
    ns = np.array([b["Mss"].shape[0] for b in blocks])
    ng = blocks[0]["Bgs"].shape[0]
    s_off = np.concatenate([[0], np.cumsum(ns)])
    nS = int(s_off[-1])
    nG = E * ng
    nU = sp.n_dof
    nH = n_uhat(sp)
    oG, oU, oH = nS, nS + nG, nS + nG + nU
    ntot = oH + nH
    hg = uhat_gdof(sp)
    rows, cols, vals = [], [], []

    def add(r_idx, c_idx, blk, sym):
        rr = np.broadcast_to(r_idx[:, None], blk.shape)
        cc = np.broadcast_to(c_idx[None, :], blk.shape)
        m = (rr >= 0) & (cc >= 0)
        rows.append(rr[m]); cols.append(cc[m]); vals.append(blk[m])
        if sym:
            rows.append(cc[m]); cols.append(rr[m]); vals.append(blk[m])

    for T, b in enumerate(blocks):
        si = s_off[T] + np.arange(ns[T])
        gi = oG + T * ng + np.arange(ng)
        ug = sp.gdof[T]
        ui = np.where(ug >= 0, oU + ug, -1)
        hi = np.where(hg[T] >= 0, oH + hg[T], -1)
        add(si, si, b["Mss"], False)
        add(gi, si, b["Bgs"], True)
        add(ui, si, b["Bus"], True)
        add(hi, si, b["Bhs"], True)
    M = mass_matrix(sp)
    Mc = M.tocoo()
    rows.append(oU + Mc.row); cols.append(oU + Mc.col); vals.append(Mc.data / dt)
    K = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(ntot, ntot)).tocsc()
    rhs = np.zeros(ntot)
    rhs[oU:oH] = M @ un / dt - (0.0 if r is None else r)
    sol = spla.spsolve(K, rhs)
    sig = [sol[s_off[T]:s_off[T + 1]] for T in range(E)]
    gam = sol[oG:oU].reshape(E, ng)
    return sol[oU:oH], sol[oH:], sig, gam, blocks


def sigma_at(sp, blocks, sig, T, ref_pts):
    """sigma of element T at reference points [N][d] -> [N][d][d]."""
    t = sp.topo
    d, k = sp.dim, sp.k
    b = blocks[T]
    mv, _ = _monomials(d, k + 1, np.atleast_2d(ref_pts) - b["xc"])
    coef = (b["N"] @ sig[T]).reshape(len(tracefree_basis(d)), -1)  # [a][m]
    return np.einsum("aij,qm,am->qij", tracefree_basis(d), mv, coef)


# ----------------------------------------------------------- condensation
def schur_system(sp, nu, dt, blocks=None):
    """S = A - B M^-1 B^t on (u, u^) (section 2.3), assembled from the
    element blocks S_T = A_T - B_T M_T^-1 B_T^t, M_T = [[Mss, Bgs^t], [Bgs, 0]],
    B_T = [[Bus, 0], [Bhs, 0]], A_T = [[M_uT/dt, 0], [0, 0]].  Returns
    (S csr, list of S_T on the element's local (u, u^) unknowns, local->global
    index [E][n + nh] with -1 for wall unknowns, blocks)."""
    t = sp.topo
    E = t.n_elems
    blocks = blocks or all_blocks(sp, nu)
    hg = uhat_gdof(sp)
    nU = sp.n_dof
    ntot = nU + n_uhat(sp)
    loc = np.concatenate([sp.gdof, np.where(hg >= 0, nU + hg, -1)], 1)
    rows, cols, vals, ST = [], [], [], []
    with threadpool_limits(1):
        ST = [_schur_block(sp, b, T, dt, hg.shape[1]) for T, b in enumerate(blocks)]
    for T, S_T in enumerate(ST):
        g = loc[T]
        rr = np.broadcast_to(g[:, None], S_T.shape)
        cc = np.broadcast_to(g[None, :], S_T.shape)
        m = (rr >= 0) & (cc >= 0)
        rows.append(rr[m]); cols.append(cc[m]); vals.append(S_T[m])
    S = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(ntot, ntot)).tocsr()
    return S, ST, loc, blocks


def _schur_block(sp, b, T, dt, nh):
    ng = b["Bgs"].shape[0]
    Mt = np.block([[b["Mss"], b["Bgs"].T], [b["Bgs"], np.zeros((ng, ng))]])
    Bt = np.concatenate([np.concatenate([b["Bus"], b["Bhs"]]),
                         np.zeros((sp.n + nh, ng))], 1)
    At = np.zeros((Bt.shape[0], Bt.shape[0]))
    At[:sp.n, :sp.n] = _mass_local(sp, T) / dt
    S_T = At - Bt @ np.linalg.solve(Mt, Bt.T)
    return 0.5 * (S_T + S_T.T)


def step_rhs(sp, un, dt, r=None):
    from .operator import mass_matrix
    f = np.zeros(sp.n_dof + n_uhat(sp))
    f[:sp.n_dof] = mass_matrix(sp) @ un / dt - (0.0 if r is None else r)
    return f


def step1_condensed(sp, un, nu, dt, r=None, schur=None):
    """(u*, u^) from S [u*; u^] = [M u^n/dt - r; 0] (direct sparse solve)."""
    S = (schur or schur_system(sp, nu, dt))[0]
    x = spla.spsolve(S.tocsc(), step_rhs(sp, un, dt, r))
    return x[:sp.n_dof], x[sp.n_dof:]


def bddc_weights(sp, loc):
    """1/2 on the broken copies of facet unknowns (u facet DoFs and u^), 1 on
    element-interior u DoFs, 0 on wall unknowns."""
    w = np.where(loc >= 0, 0.5, 0.0)
    r0 = (sp.dim + 1) * sp.nf
    w[:, r0:sp.n] = 1.0
    return w


def bddc_apply(sp, schur, x):
    """C^-1 x = R S_BDDC^-1 R^t x with S_BDDC = blockdiag(S_T) on the broken
    space (section 2.3): each element solves with its own S_T on its non-wall
    unknowns; R averages the two copies of every facet unknown."""
    _, ST, loc, _ = schur
    w = bddc_weights(sp, loc)
    z = np.zeros_like(x)
    for T, S_T in enumerate(ST):
        g = loc[T]
        m = g >= 0
        xt = w[T][m] * x[g[m]]
        yt = np.linalg.solve(S_T[np.ix_(m, m)], xt)
        np.add.at(z, g[m], w[T][m] * yt)
    return z


def step1_pcg(sp, un, nu, dt, r=None, rtol=1e-12, max_it=2000, schur=None):
    """The paper's solver: PCG on S with the element-wise BDDC C^-1, zero
    initial guess.  Returns (u*, u^, iterations)."""
    schur = schur or schur_system(sp, nu, dt)
    S = schur[0]
    b = step_rhs(sp, un, dt, r)
    x = np.zeros_like(b)
    res = b.copy()
    z = bddc_apply(sp, schur, res)
    p = z.copy()
    rz = res @ z
    tol = rtol * np.sqrt(abs(rz))
    it = 0
    while it < max_it and np.sqrt(abs(rz)) > tol:
        q = S @ p
        a = rz / (p @ q)
        x += a * p
        res -= a * q
        z = bddc_apply(sp, schur, res)
        rz_new = res @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x[:sp.n_dof], x[sp.n_dof:], it


def viscous_energy(blocks, sig, nu):
    """||sigma||^2 / (2 nu) = -a(sigma, sigma)."""
    return -sum(s @ b["Mss"] @ s for b, s in zip(blocks, sig))
