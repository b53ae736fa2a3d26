"""Projection step of the operator splitting (paper section 2.3, eq.
(MCS_step2) and the update eq. (UpdateStep)); oracle, test infrastructure
only.

Given u* in V_h, find (u~, p, p^) in V_h^disc x Q_h x Q^_h with
    -(u~, v~) + b1(v~, p) + b3(v~, p^) = 0           for all v~ in V_h^disc
     b1(u~, q) + b3(u~, q^)            = b1(u*, q)   for all (q, q^)
where
    V_h^disc  the element-wise (broken) velocity space: on each element the
              same local space and dual basis as V_h, without continuity;
    Q_h       = div V_h = P^{k-1} per element (the paper's compatibility
              condition div V_h in Q_h; with BDM_k this is P^{k-1});
    Q^_h      = P^k on every facet, walls included (no Neumann facets in
              these workloads);
    b1(v, q)  = -sum_T int_T (div v) q;
    b3(v, q^) = sum_T int_{dT} (v . n_T) q^.
The update is u^{n+1} = u* - u~ (the reading of eq. (UpdateStep) used here:
the Chorin projection, whose divergence-free proof only uses
div(u* - u~) = 0).

Bases.  V_h^disc uses the physical dual basis of each element (global DoF
T * n + i).  Q_h uses the reference scalar basis of degree k-1 mapped by
the affine map.  On a facet F with unit normal n_F and parametrisation
x_F(s) (|dx/ds| = |N_F|), Q^_h uses psi~_{F,j}(x) = psi_j(s(x)) / |N_F|, so
that int_F (v . n_F) psi~_{F,j} = x_{F,j}(v), the facet DoF: b3 of a local
basis function against psi~_{F,j} is sigma_{T,F} (the outward sign of n_F
for T) when it is that facet DoF, else 0.

The saddle-point system is solved directly (sparse LU).  (p, p^) = (c, c)
is in its kernel (b1(v, c) + b3(v, c) = 0 by the divergence theorem), so
the constant mode of p^ on the first facet is fixed to zero; u~ does not
depend on that choice.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from . import basis as B


def _wall_facets(t):
    """(element, local facet) of every wall facet, in the order of
    topo.wall_elems / wall_local."""
    return np.asarray(t.wall_elems, dtype=np.int64), np.asarray(t.wall_local, dtype=np.int64)


def facet_multiplier_index(sp):
    """[E][d+1] index of the Q^_h facet block of each element facet:
    interior facets first (their global facet index), then wall facets."""
    t = sp.topo
    idx = np.array(t.elem_facet, dtype=np.int64)
    we, wl = _wall_facets(t)
    idx[we, wl] = t.n_facets + np.arange(len(we))
    return idx, t.n_facets + len(we)


def local_blocks(sp, elems):
    """Per element: M_T [n][n], B_T [nQ][n] (b1 of the local basis against
    the Q_h basis)."""
    t = sp.topo
    phi = sp.phys_vals(elems, sp.ref_vals)                  # [b][q][n][d]
    gphi = sp.phys_grads(elems, sp.ref_grads)               # [b][q][n][d][d]
    wdx = sp.wq[None, :] * np.abs(t.detJ[elems])[:, None]   # [b][q]
    M = np.einsum("bq,bqid,bqjd->bij", wdx, phi, phi)
    div = np.einsum("bqiaa->bqi", gphi)
    q = B.scalar_basis(sp.dim, sp.k - 1, sp.xq)[0]
    Bt = -np.einsum("bq,bqi,qm->bmi", wdx, div, q)
    return M, Bt


def n_pressure(sp):
    return B.dim_P(sp.dim, sp.k - 1)


def project(sp, ustar):
    """(u_new, u_tilde_broken [E][n], p [E][nQ], p_hat [nFq][nf]) for u* in
    V_h; u_new = u* - u~ in the V_h coefficient layout."""
    t = sp.topo
    E, n, d, nf = t.n_elems, sp.n, sp.dim, sp.nf
    nQ = n_pressure(sp)
    fidx, nFq = facet_multiplier_index(sp)
    Ms, Bs = [], []
    for eb in sp.batches(E, max(1, sp.elem_batch_size())):
        M, Bt = local_blocks(sp, eb)
        Ms.append(M)
        Bs.append(Bt)
    M = np.concatenate(Ms)
    Bt = np.concatenate(Bs)
    nU, nP, nH = E * n, E * nQ, nFq * nf
    e_idx = np.arange(E)
    # -M (block diagonal)
    r = (e_idx[:, None, None] * n + np.arange(n)[None, :, None]).repeat(n, 2)
    c = (e_idx[:, None, None] * n + np.arange(n)[None, None, :]).repeat(n, 1)
    Mb = sps.coo_matrix((-M.ravel(), (r.ravel(), c.ravel())), shape=(nU, nU))
    # B: rows p (E*nQ), cols u~
    rb = (e_idx[:, None, None] * nQ + np.arange(nQ)[None, :, None]).repeat(n, 2)
    cb = (e_idx[:, None, None] * n + np.arange(n)[None, None, :]).repeat(nQ, 1)
    Bb = sps.coo_matrix((Bt.ravel(), (rb.ravel(), cb.ravel())), shape=(nP, nU))
    # C: rows p^ (facet block, nf each), cols u~: sigma on the facet DoF
    rc, cc, vc = [], [], []
    for i in range(d + 1):
        for j in range(nf):
            rc.append(fidx[:, i] * nf + j)
            cc.append(e_idx * n + i * nf + j)
            vc.append(np.asarray(t.sigma[:, i], dtype=float))
    Cb = sps.coo_matrix((np.concatenate(vc), (np.concatenate(rc), np.concatenate(cc))), shape=(nH, nU))
    K = sps.bmat([[Mb, Bb.T, Cb.T], [Bb, None, None], [Cb, None, None]], format="csr")
    # right-hand side: b1(u*, q)
    ub = sp.local(ustar, e_idx)                            # [E][n] (0 on wall DoFs)
    rhs = np.zeros(nU + nP + nH)
    rhs[nU:nU + nP] = np.einsum("emi,ei->em", Bt, ub).ravel()
    # fix the kernel: p^ constant mode (psi_0) of multiplier block 0
    keep = np.ones(K.shape[0], dtype=bool)
    keep[nU + nP + 0] = False
    sol = np.zeros(K.shape[0])
    Kk = K[keep][:, keep].tocsc()
    sol[keep] = spla.spsolve(Kk, rhs[keep])
    ut = sol[:nU].reshape(E, n)
    p = sol[nU:nU + nP].reshape(E, nQ)
    ph = sol[nU + nP:].reshape(nFq, nf)
    # u~ is normal-continuous: read it in the V_h layout (facet DoFs from
    # the lower-id neighbour, interior DoFs from their element)
    ut_h = np.zeros(sp.n_dof)
    g = sp.gdof
    for ee in (e_idx[::-1],):  # lower element ids written last
        m = g[ee] >= 0
        ut_h[g[ee][m]] = ut[ee][m]
    return ustar - ut_h, ut, p, ph


def normal_jump(sp, ut):
    """max |x_T - x_T'| over the shared facet DoFs of a broken field, and
    max |x_T| over wall facet DoFs (both zero for u~ in V_h)."""
    t = sp.topo
    nf = sp.nf
    j = 0.0
    for F in range(t.n_facets):
        (T, T2), (i, i2) = t.facet_elems[F], t.facet_local[F]
        j = max(j, float(np.abs(ut[T, i * nf:(i + 1) * nf] - ut[T2, i2 * nf:(i2 + 1) * nf]).max()))
    w = 0.0
    we, wl = _wall_facets(t)
    for T, i in zip(we, wl):
        w = max(w, float(np.abs(ut[T, i * nf:(i + 1) * nf]).max()))
    return j, w


def projection_dense(sp, ustar):
    """The M-orthogonal projection of u* onto {v in V_h : b1(v, q) = 0 for
    all q in Q_h}, written without hybridisation (dense; tiny meshes only):
    u_new = u* - M^-1 B^t lambda with (B M^-1 B^t) lambda = B u*."""
    from .operator import mass_matrix
    t = sp.topo
    E, n = t.n_elems, sp.n
    nQ = n_pressure(sp)
    M = mass_matrix(sp).toarray()
    Bg = np.zeros((E * nQ, sp.n_dof))
    for eb in sp.batches(E, max(1, sp.elem_batch_size())):
        _, Bt = local_blocks(sp, eb)
        for a, e in enumerate(eb):
            g = sp.gdof[e]
            m = g >= 0
            Bg[e * nQ:(e + 1) * nQ, g[m]] += Bt[a][:, m]
    Minv_Bt = np.linalg.solve(M, Bg.T)
    S = Bg @ Minv_Bt
    lam = np.linalg.lstsq(S, Bg @ ustar, rcond=None)[0]
    return ustar - Minv_Bt @ lam
