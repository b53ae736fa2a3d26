"""The HOPU convection operator, mass matrix, substeps, diagnostics and
adjoints (oracle; test infrastructure only).  Plain definitions evaluated in
physical coordinates, element and facet loops vectorised over batches.

Residual (conservative volume form; the paper writes the volume term in the
advective form (grad u u) . v, eq. (upwind) and eq. (hopudefinition); the two
differ by -sum_T int (div u)(u . v), zero for divergence-free u):

  r_i(u) = - sum_T int_T (u x u) : grad phi_i dx
           + sum_{E in F^I} int_E (u.n) <u> . [[phi_i]]
                              + 1/2 |u.n| (I - Pi^l)[[u]] . (I - Pi^l)[[phi_i]] ds

with (a x b):grad v = sum a_i b_j d_j v_i, n the outward normal of the element
called T, [[f]] = f^T - f^T', <f> = (f^T + f^T')/2 (section 2.1) and Pi^l the
facet-wise L2 projection onto polynomials of degree <= l computed with the
facet rule (section 3.2); l = -1 means Pi = 0 (standard upwind, eq. (upwind)),
l = k means Pi = I (central flux).
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

TERM_VOLUME, TERM_CENTRAL, TERM_UPWIND = 1, 2, 4
TERM_ALL = 7


# ------------------------------------------------------------------ facets
def _facet_batches(sp, size=2048, facets=None):
    t = sp.topo
    if facets is not None:
        for s in range(0, len(facets), size):
            yield facets[s:s + size]
        return
    for s in range(0, t.n_facets, size):
        yield np.arange(s, min(t.n_facets, s + size))


def _elem_batches(sp, elems, size):
    if elems is None:
        yield from sp.batches(sp.topo.n_elems, size)
        return
    for s in range(0, len(elems), size):
        yield elems[s:s + size]


def _facets_of(sp, elems):
    """Interior facets touching the given elements (sorted)."""
    if elems is None:
        return None
    f = sp.topo.elem_facet[elems].ravel()
    return np.unique(f[f >= 0])


def _facet_traces(sp, fb):
    """Physical basis traces of both neighbours at the facet points and
    the facet geometry: phiT, phiT2 [B][nqf][n][d], n [B][d], ds [B][nqf]."""
    t = sp.topo
    T, T2 = t.facet_elems[fb, 0], t.facet_elems[fb, 1]
    i, i2 = t.facet_local[fb, 0], t.facet_local[fb, 1]
    phiT = np.empty((len(fb), len(sp.wsq), sp.n, sp.dim))
    phiT2 = np.empty_like(phiT)
    for loc in range(sp.dim + 1):
        m = i == loc
        if m.any():
            phiT[m] = sp.phys_vals(T[m], sp.ref_face[loc])
        m = i2 == loc
        if m.any():
            phiT2[m] = sp.phys_vals(T2[m], sp.ref_face[loc])
    nvec = (t.sigma[T, i] / t.NF_norm[T, i])[:, None] * t.NF[T, i]
    ds = t.NF_norm[T, i][:, None] * sp.wsq[None, :]
    return T, T2, phiT, phiT2, nvec, ds


def _projector(sp, lf):
    """Matrices P_f [B][nqf][nqf] of the discrete L2 projection onto facet
    polynomials of degree <= l_f:  (P f)_q = sum_{deg psi_j <= l} psi_j(q)
    sum_q' w_q' psi_j(q') f_q'."""
    psi, w = sp.psi_q, sp.wsq
    mask = (sp.psi_deg[None, :] <= lf[:, None]).astype(float)  # [B][nf]
    return np.einsum("qj,bj,pj,p->bqp", psi, mask, psi, w)


def residual(sp, x, l, terms=TERM_ALL, elems=None):
    """elems (optional): evaluate only the volume terms of these elements and
    the facet terms of their facets; rows of their interior DoFs, and of
    facets whose two elements are both listed, are then complete."""
    t = sp.topo
    r = np.zeros(sp.n_dof)
    if terms & TERM_VOLUME:
        for eb in _elem_batches(sp, elems, sp.elem_batch_size()):
            xl = sp.local(x, eb)
            phi = sp.phys_vals(eb, sp.ref_vals)
            gphi = sp.phys_grads(eb, sp.ref_grads)
            u = np.einsum("bqid,bi->bqd", phi, xl)
            wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
            val = np.einsum("bq,bqa,bqc,bqiac->bi", wdx, u, u, gphi)
            sp.scatter(r, eb, -val)
    if terms & (TERM_CENTRAL | TERM_UPWIND):
        lf_all = sp.facet_l(l)
        for fb in _facet_batches(sp, facets=_facets_of(sp, elems)):
            T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
            uT = np.einsum("bqid,bi->bqd", phiT, sp.local(x, T))
            uT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(x, T2))
            avg = 0.5 * (uT + uT2)
            jump = uT - uT2
            un = np.einsum("bqd,bd->bq", avg, nvec)
            rT = np.zeros((len(fb), sp.n))
            rT2 = np.zeros((len(fb), sp.n))
            if terms & TERM_CENTRAL:
                g = un[:, :, None] * avg
                rT += np.einsum("bq,bqd,bqid->bi", ds, g, phiT)
                rT2 -= np.einsum("bq,bqd,bqid->bi", ds, g, phiT2)
            if terms & TERM_UPWIND:
                P = _projector(sp, lf_all[fb])
                jp = jump - np.einsum("bqp,bpd->bqd", P, jump)
                tT = phiT - np.einsum("bqp,bpid->bqid", P, phiT)    # (I-Pi) phi^T
                tT2 = phiT2 - np.einsum("bqp,bpid->bqid", P, phiT2)
                a = 0.5 * np.abs(un) * ds
                rT += np.einsum("bq,bqd,bqid->bi", a, jp, tT)
                rT2 -= np.einsum("bq,bqd,bqid->bi", a, jp, tT2)
            sp.scatter(r, T, rT)
            sp.scatter(r, T2, rT2)
    return r


def residual_advective(sp, x, l, upwind=True):
    """The paper's form, eq. (hopudefinition):
    sum_T int (grad u u).v - sum_E int (u.n)[[u]].<v> + upwind term."""
    t = sp.topo
    r = np.zeros(sp.n_dof)
    for eb in sp.batches(t.n_elems, sp.elem_batch_size()):
        xl = sp.local(x, eb)
        phi = sp.phys_vals(eb, sp.ref_vals)
        gphi = sp.phys_grads(eb, sp.ref_grads)
        u = np.einsum("bqid,bi->bqd", phi, xl)
        gu = np.einsum("bqiac,bi->bqac", gphi, xl)   # d_c u_a
        conv = np.einsum("bqac,bqc->bqa", gu, u)
        wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
        sp.scatter(r, eb, np.einsum("bq,bqa,bqia->bi", wdx, conv, phi))
    lf_all = sp.facet_l(l)
    for fb in _facet_batches(sp):
        T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
        uT = np.einsum("bqid,bi->bqd", phiT, sp.local(x, T))
        uT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(x, T2))
        jump = uT - uT2
        un = np.einsum("bqd,bd->bq", 0.5 * (uT + uT2), nvec)
        g = -(un * ds)[:, :, None] * jump
        rT = 0.5 * np.einsum("bqd,bqid->bi", g, phiT)
        rT2 = 0.5 * np.einsum("bqd,bqid->bi", g, phiT2)
        if upwind:
            P = _projector(sp, lf_all[fb])
            jp = jump - np.einsum("bqp,bpd->bqd", P, jump)
            tT = phiT - np.einsum("bqp,bpid->bqid", P, phiT)
            tT2 = phiT2 - np.einsum("bqp,bpid->bqid", P, phiT2)
            a = 0.5 * np.abs(un) * ds
            rT += np.einsum("bq,bqd,bqid->bi", a, jp, tT)
            rT2 -= np.einsum("bq,bqd,bqid->bi", a, jp, tT2)
        sp.scatter(r, T, rT)
        sp.scatter(r, T2, rT2)
    return r


# ------------------------------------------------------------------ mass
def mass_matrix(sp):
    """M_ij = int phi_i . phi_j (the paper's M_uu = M / dt, section 2.3)."""
    cache = getattr(sp, "_mass", None)
    if cache is not None:
        return cache
    t = sp.topo
    rows, cols, vals = [], [], []
    for eb in sp.batches(t.n_elems, max(1, sp.elem_batch_size() * sp.dim)):
        phi = sp.phys_vals(eb, sp.ref_vals)
        wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
        Me = np.einsum("bq,bqid,bqjd->bij", wdx, phi, phi)
        g = sp.gdof[eb]
        gi = np.broadcast_to(g[:, :, None], Me.shape)
        gj = np.broadcast_to(g[:, None, :], Me.shape)
        m = (gi >= 0) & (gj >= 0)
        rows.append(gi[m])
        cols.append(gj[m])
        vals.append(Me[m])
    M = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                        np.concatenate(cols))), shape=(sp.n_dof, sp.n_dof)).tocsr()
    sp._mass = M
    return M


def mass_solve(sp, r, method=None):
    """w = M^{-1} r: sparse LU for small spaces, CG to 1e-15 otherwise.
    method "cg" asks for the CG solve at any size (the LU's fill on large 3D
    meshes costs minutes; CG reaches relative residuals near 1e-13 there,
    enough for convergence-order checks, not for 1e-12 parity)."""
    M = mass_matrix(sp)
    if sp.n_dof <= 200000 and method != "cg":
        lu = getattr(sp, "_mass_lu", None)
        if lu is None:
            lu = spla.splu(M.tocsc())
            sp._mass_lu = lu
        return lu.solve(r)
    d = M.diagonal()
    pre = spla.LinearOperator(M.shape, matvec=lambda v: v / d)
    w, info = spla.cg(M, r, rtol=1e-15, atol=0.0, maxiter=5000, M=pre)
    if info != 0:
        raise RuntimeError("oracle CG did not converge")
    return w


# ------------------------------------------------------------ substeps
def substep(sp, x, dt, l):
    """u <- u - dt M^{-1} r(u): the explicit convection part of step 1
    (eq. (MCS_step1) with M_uu = M/dt)."""
    return x - dt * mass_solve(sp, residual(sp, x, l))


def substeps(sp, x0, dt, n_steps, l, keep=False):
    xs = [x0]
    x = x0
    for _ in range(n_steps):
        x = substep(sp, x, dt, l)
        if keep:
            xs.append(x)
    return xs if keep else x


# ------------------------------------------------------------ diagnostics
def energy(sp, x):
    return 0.5 * float(x @ (mass_matrix(sp) @ x))


def divergence_l2(sp, x):
    t = sp.topo
    acc = 0.0
    for eb in sp.batches(t.n_elems, sp.elem_batch_size()):
        gphi = sp.phys_grads(eb, sp.ref_grads)
        gu = np.einsum("bqiac,bi->bqac", gphi, sp.local(x, eb))
        div = np.einsum("bqaa->bq", gu)
        acc += float(np.sum(sp.wq[None, :] * np.abs(t.detJ[eb])[:, None] * div ** 2))
    return np.sqrt(acc)


def dissipation(sp, x, l):
    """D = sum_E int_E 1/2 |u.n| |(I - Pi^l)[[u]]|^2 ds."""
    lf_all = sp.facet_l(l)
    acc = 0.0
    for fb in _facet_batches(sp):
        T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
        uT = np.einsum("bqid,bi->bqd", phiT, sp.local(x, T))
        uT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(x, T2))
        jump = uT - uT2
        un = np.einsum("bqd,bd->bq", 0.5 * (uT + uT2), nvec)
        P = _projector(sp, lf_all[fb])
        jp = jump - np.einsum("bqp,bpd->bqd", P, jump)
        acc += float(np.sum(0.5 * np.abs(un) * ds * np.sum(jp ** 2, -1)))
    return acc


# ------------------------------------------------------------ adjoints
SGN_ZERO_TOL = 1e-8


def sgn0(un, avg):
    """The derivative of |u.n| with sgn(0) := 0, where "0" is any u.n within
    SGN_ZERO_TOL |<u>| of zero: u.n that vanishes in exact arithmetic (a field
    tangential to a facet) is rounding noise of either sign, and its sign
    would decide an O(1) term.  Two FP64 ways of evaluating u.n (the average
    of the traces, the facet DoFs' polynomial) differ by up to about 1e-11
    |<u>| at k <= 5, while u.n that does not vanish is far above 1e-8 |<u>|
    on the smooth fields of the convection tests."""
    scale = np.sqrt(np.sum(avg * avg, -1))
    return np.where(np.abs(un) <= SGN_ZERO_TOL * scale, 0.0, np.sign(un))


def vjp(sp, x, mu, l, elems=None):
    """(J_r(u)^T mu)_j = d/du_j sum_i mu_i r_i(u), with mu_h = sum mu_i phi_i:
      - sum_T int phi_j . (grad mu_h + grad mu_h^T) u
      + sum_E int (phi_j.n) s + (u.n) <phi_j>.[[mu_h]]
                  + 1/2 |u.n| (I-Pi)[[phi_j]] . (I-Pi)[[mu_h]]
      s = <u>.[[mu_h]] + 1/2 sgn(u.n) (I-Pi)[[u]] . (I-Pi)[[mu_h]], sgn(0) = 0
          (sgn0: u.n within 1e-8 |<u>| of zero counts as zero);
    phi_j . n is single valued and equals <phi_j> . n.  `elems` restricts the
    loops as in residual()."""
    t = sp.topo
    out = np.zeros(sp.n_dof)
    for eb in _elem_batches(sp, elems, sp.elem_batch_size()):
        phi = sp.phys_vals(eb, sp.ref_vals)
        gphi = sp.phys_grads(eb, sp.ref_grads)
        u = np.einsum("bqid,bi->bqd", phi, sp.local(x, eb))
        gm = np.einsum("bqiac,bi->bqac", gphi, sp.local(mu, eb))  # d_c mu_a
        v = np.einsum("bqac,bqc->bqa", gm, u) + np.einsum("bqca,bqc->bqa", gm, u)
        wdx = sp.wq[None, :] * np.abs(t.detJ[eb])[:, None]
        sp.scatter(out, eb, -np.einsum("bq,bqa,bqia->bi", wdx, v, phi))
    lf_all = sp.facet_l(l)
    for fb in _facet_batches(sp, facets=_facets_of(sp, elems)):
        T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
        uT = np.einsum("bqid,bi->bqd", phiT, sp.local(x, T))
        uT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(x, T2))
        mT = np.einsum("bqid,bi->bqd", phiT, sp.local(mu, T))
        mT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(mu, T2))
        avg = 0.5 * (uT + uT2)
        un = np.einsum("bqd,bd->bq", avg, nvec)
        P = _projector(sp, lf_all[fb])
        ju = uT - uT2
        jm = mT - mT2
        jup = ju - np.einsum("bqp,bpd->bqd", P, ju)
        jmp = jm - np.einsum("bqp,bpd->bqd", P, jm)
        s = np.sum(avg * jm, -1) + 0.5 * sgn0(un, avg) * np.sum(jup * jmp, -1)
        tT = phiT - np.einsum("bqp,bpid->bqid", P, phiT)
        tT2 = phiT2 - np.einsum("bqp,bpid->bqid", P, phiT2)
        phin_T = np.einsum("bqid,bd->bqi", phiT, nvec)
        phin_T2 = np.einsum("bqid,bd->bqi", phiT2, nvec)
        rT = 0.5 * np.einsum("bq,bqi->bi", ds * s, phin_T)
        rT2 = 0.5 * np.einsum("bq,bqi->bi", ds * s, phin_T2)
        rT += 0.5 * np.einsum("bq,bqd,bqid->bi", ds * un, jm, phiT)
        rT2 += 0.5 * np.einsum("bq,bqd,bqid->bi", ds * un, jm, phiT2)
        a = 0.5 * np.abs(un) * ds
        rT += np.einsum("bq,bqd,bqid->bi", a, jmp, tT)
        rT2 -= np.einsum("bq,bqd,bqid->bi", a, jmp, tT2)
        sp.scatter(out, T, rT)
        sp.scatter(out, T2, rT2)
    return out


def mass_apply(sp, x):
    return mass_matrix(sp) @ x


def chain_vjp(sp, x0, dt, n_steps, l, lam_N):
    """Reverse pass of u_{n+1} = u_n - dt M^{-1} r(u_n):
    lam_n = lam_{n+1} - dt J_r(u_n)^T M^{-1} lam_{n+1}; returns lam_0."""
    xs = substeps(sp, x0, dt, n_steps, l, keep=True)
    lam = lam_N.copy()
    for s in range(n_steps - 1, -1, -1):
        mu = mass_solve(sp, lam)
        lam = lam - dt * vjp(sp, xs[s], mu, l)
    return lam


# ------------------------------------------------------ assembled matrices
def assemble_picard(sp, w, l, terms=TERM_ALL):
    """Dense C(w)_ij = c(w; phi_j, phi_i): the residual's bilinear form with
    convecting field w (reading of the garbled C_uu, section 2.3), built by
    double loops over physical basis products.  Tiny meshes only."""
    t = sp.topo
    N = sp.n_dof
    C = np.zeros((N, N))
    for e in range(t.n_elems):
        eb = np.array([e])
        phi = sp.phys_vals(eb, sp.ref_vals)[0]
        gphi = sp.phys_grads(eb, sp.ref_grads)[0]
        u = np.einsum("qid,i->qd", phi, sp.local(w, eb)[0])
        wdx = sp.wq * abs(t.detJ[e])
        g = sp.gdof[e]
        if terms & TERM_VOLUME:
            for a_ in range(sp.n):
                for b_ in range(sp.n):
                    if g[a_] < 0 or g[b_] < 0:
                        continue
                    # -int (phi_j x u) : grad phi_i
                    v = -np.sum(wdx * np.einsum("qa,qc,qac->q", phi[:, b_], u, gphi[:, a_]))
                    C[g[a_], g[b_]] += v
    lf_all = sp.facet_l(l)
    for f in range(t.n_facets):
        fb = np.array([f])
        T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
        phiT, phiT2, nvec, ds = phiT[0], phiT2[0], nvec[0], ds[0]
        uT = np.einsum("qid,i->qd", phiT, sp.local(w, T)[0])
        uT2 = np.einsum("qid,i->qd", phiT2, sp.local(w, T2)[0])
        un = (0.5 * (uT + uT2)) @ nvec
        P = _projector(sp, lf_all[fb])[0]
        gT, gT2 = sp.gdof[T[0]], sp.gdof[T2[0]]
        # basis functions as global functions on the facet: jump / average
        idx = sorted(set(gT[gT >= 0]) | set(gT2[gT2 >= 0]))
        tr1, tr2 = {}, {}
        for gg in idx:
            a1 = np.zeros((len(ds), sp.dim))
            a2 = np.zeros((len(ds), sp.dim))
            for loc in np.nonzero(gT == gg)[0]:
                a1 += phiT[:, loc]
            for loc in np.nonzero(gT2 == gg)[0]:
                a2 += phiT2[:, loc]
            tr1[gg], tr2[gg] = a1, a2
        for gi in idx:
            ji = tr1[gi] - tr2[gi]
            jip = ji - P @ ji
            for gj in idx:
                aj = 0.5 * (tr1[gj] + tr2[gj])
                jj = tr1[gj] - tr2[gj]
                jjp = jj - P @ jj
                v = 0.0
                if terms & TERM_CENTRAL:
                    v += np.sum(ds * un * np.sum(aj * ji, -1))
                if terms & TERM_UPWIND:
                    v += np.sum(ds * 0.5 * np.abs(un) * np.sum(jjp * jip, -1))
                C[gi, gj] += v
    return C


def assemble_jacobian(sp, w, l, terms=TERM_ALL):
    """Dense Jacobian J(w)_ij = d r_i / d u_j at u = w, by double loops over
    physical basis products of the linearised residual (tiny meshes only).
    Differentiating each term of the residual in the direction phi_j:
      volume   - int (phi_j x w + w x phi_j) : grad phi_i
      central  + int (<phi_j>.n) <w>.[[phi_i]] + (w.n) <phi_j>.[[phi_i]]
      upwind   + int 1/2 sgn(w.n) (<phi_j>.n) (I-Pi)[[w]] . (I-Pi)[[phi_i]]
                     + 1/2 |w.n| (I-Pi)[[phi_j]] . (I-Pi)[[phi_i]]
    with sgn(0) = 0 (|.| is not differentiable at 0; the reading used for
    the adjoint), u.n within 1e-8 |<w>| of zero counting as zero (sgn0).
    Written independently of vjp(): J^T mu must equal vjp(w, mu), and
    J(w) w = 2 r(w) (r is homogeneous of degree 2)."""
    t = sp.topo
    N = sp.n_dof
    Jm = np.zeros((N, N))
    if terms & TERM_VOLUME:
        for e in range(t.n_elems):
            eb = np.array([e])
            phi = sp.phys_vals(eb, sp.ref_vals)[0]      # [q][n][d]
            gphi = sp.phys_grads(eb, sp.ref_grads)[0]   # [q][n][a][c] = d_c phi_a
            u = np.einsum("qid,i->qd", phi, sp.local(w, eb)[0])
            wdx = sp.wq * abs(t.detJ[e])
            g = sp.gdof[e]
            for a_ in range(sp.n):
                if g[a_] < 0:
                    continue
                for b_ in range(sp.n):
                    if g[b_] < 0:
                        continue
                    pj = phi[:, b_]
                    # (phi_j x w + w x phi_j) : grad phi_i, sum over a, c
                    v = np.einsum("qa,qc,qac->q", pj, u, gphi[:, a_]) + \
                        np.einsum("qa,qc,qac->q", u, pj, gphi[:, a_])
                    Jm[g[a_], g[b_]] -= np.sum(wdx * v)
    if terms & (TERM_CENTRAL | TERM_UPWIND):
        lf_all = sp.facet_l(l)
        for f in range(t.n_facets):
            fb = np.array([f])
            T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
            phiT, phiT2, nvec, ds = phiT[0], phiT2[0], nvec[0], ds[0]
            wT = np.einsum("qid,i->qd", phiT, sp.local(w, T)[0])
            wT2 = np.einsum("qid,i->qd", phiT2, sp.local(w, T2)[0])
            wavg = 0.5 * (wT + wT2)
            wn = wavg @ nvec
            P = _projector(sp, lf_all[fb])[0]
            wjp = (wT - wT2) - P @ (wT - wT2)
            gT, gT2 = sp.gdof[T[0]], sp.gdof[T2[0]]
            idx = sorted(set(gT[gT >= 0]) | set(gT2[gT2 >= 0]))
            tr1, tr2 = {}, {}
            for gg in idx:
                a1 = np.zeros((len(ds), sp.dim))
                a2 = np.zeros((len(ds), sp.dim))
                for loc in np.nonzero(gT == gg)[0]:
                    a1 += phiT[:, loc]
                for loc in np.nonzero(gT2 == gg)[0]:
                    a2 += phiT2[:, loc]
                tr1[gg], tr2[gg] = a1, a2
            for gi in idx:
                ji = tr1[gi] - tr2[gi]
                jip = ji - P @ ji
                for gj in idx:
                    aj = 0.5 * (tr1[gj] + tr2[gj])
                    ajn = aj @ nvec
                    jj = tr1[gj] - tr2[gj]
                    jjp = jj - P @ jj
                    v = 0.0
                    if terms & TERM_CENTRAL:
                        v += np.sum(ds * (ajn * np.sum(wavg * ji, -1) + wn * np.sum(aj * ji, -1)))
                    if terms & TERM_UPWIND:
                        v += np.sum(ds * 0.5 * sgn0(wn, wavg) * ajn * np.sum(wjp * jip, -1))
                        v += np.sum(ds * 0.5 * np.abs(wn) * np.sum(jjp * jip, -1))
                    Jm[gi, gj] += v
    return Jm


def assemble_mass_dense(sp):
    return mass_matrix(sp).toarray()


# ------------------------------------------------------ adaptive HOPU order
def jump_indicator(sp, x, l):
    """Facet jump indicator of the adaptive HOPU order (end of section 3.2):
    eta_E = int_E |(I - Pi^l)[[u]]| ds / int_E |<u>| ds (Euclidean norms),
    evaluated with the facet rule and the facet's current l.  A facet with
    <u> = 0 everywhere gets eta = 0 if its projected jump is zero, else +inf."""
    lf_all = sp.facet_l(l)
    eta = np.empty(sp.topo.n_facets)
    for fb in _facet_batches(sp):
        T, T2, phiT, phiT2, nvec, ds = _facet_traces(sp, fb)
        uT = np.einsum("bqid,bi->bqd", phiT, sp.local(x, T))
        uT2 = np.einsum("bqid,bi->bqd", phiT2, sp.local(x, T2))
        jump = uT - uT2
        P = _projector(sp, lf_all[fb])
        jp = jump - np.einsum("bqp,bpd->bqd", P, jump)
        num = np.sum(ds * np.linalg.norm(jp, axis=-1), -1)
        den = np.sum(ds * np.linalg.norm(0.5 * (uT + uT2), axis=-1), -1)
        with np.errstate(divide="ignore", invalid="ignore"):
            e = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
        eta[fb] = e
    return eta


def adapt_order(eta, thresholds, k):
    """l_loc from eta and thresholds eta_0 < ... < eta_k (eta_{k+1} = 1):
    eta_i < eta <= eta_{i+1} gives l = i; eta <= eta_0 gives -1 (standard
    upwind); eta > 1 gives k."""
    th = list(thresholds) + [1.0]
    assert len(th) == k + 2
    out = np.full(eta.shape, -1, dtype=np.int64)
    for i in range(k + 1):
        out[(eta > th[i]) & (eta <= th[i + 1])] = i
    out[eta > 1.0] = k
    return out


def substeps_adaptive(sp, x0, dt, n_steps, thresholds, every=10, l0=-1):
    """Substeps with the adaptive order: before every `every`-th step the
    facet orders are recomputed from the jump indicator of the current state
    (evaluated with the orders in use, initially l0)."""
    l = np.full(sp.topo.n_facets, l0, dtype=np.int64)
    x = x0
    for s in range(n_steps):
        if s % every == 0:
            l = adapt_order(jump_indicator(sp, x, l), thresholds, sp.k)
        x = substep(sp, x, dt, l)
    return x, l
