"""The discrete velocity space V_h on a mesh: DoF numbering, physical basis,
interpolation and evaluation (oracle; test infrastructure only).

Coefficient convention (the paper only names a hierarchical basis, remark
in section 2.3; the reading used here is the dual basis of scaled
functionals):
  facet DoF      x_{F,j} = int_S^ (u(x_F(s)) . n_F) psi_j(s) ds
  interior DoF   x_{T,m} = |det J|^{-(d-1)/d} int_T^ (det J J^{-1} u(F_T(x^))) . q_m dx^
The physical basis is phi_{T,i} = S_ii J phi^_i(x^) / det J (signed Piola map of
the reference dual basis) with S_ii = |N_F| for facet DoFs and
|det J|^{(d-1)/d} for interior DoFs.  Normal continuity: u . n_F is the same
polynomial sum_j x_{F,j} psi_j seen from both neighbours.

Global vector layout: [interior-facet block: facets in lexicographic order,
n_f each] ++ [element-interior block: elements in input order, n_int each].
Wall facets carry no DoFs (normal velocity zero, section 2.2 remark on
boundary conditions).
"""
import numpy as np

from . import basis as B
from . import mesh as OM
from .quadrature import simplex_rule, volume_points_per_dir, facet_points_per_dir


class Space:
    def __init__(self, elem_vid, elem_xyz, k):
        self.topo = t = OM.build(elem_vid, elem_xyz)
        self.dim = d = t.dim
        self.k = k
        self.nP = B.dim_P(d, k)
        self.n = d * self.nP
        self.nf = B.n_facet_dofs(d, k)
        self.nint = B.n_interior_dofs(d, k)
        E = t.n_elems
        F = t.n_facets
        self.n_dof = F * self.nf + E * self.nint
        # element-local -> global DoF map (-1 for wall facet DoFs)
        g = -np.ones((E, self.n), dtype=np.int64)
        for i in range(d + 1):
            f = t.elem_facet[:, i]
            for j in range(self.nf):
                g[:, i * self.nf + j] = np.where(f >= 0, f * self.nf + j, -1)
        r0 = (d + 1) * self.nf
        g[:, r0:] = F * self.nf + np.arange(E)[:, None] * self.nint + np.arange(self.nint)[None, :]
        self.gdof = g
        S = np.empty((E, self.n))
        for i in range(d + 1):
            S[:, i * self.nf:(i + 1) * self.nf] = t.NF_norm[:, i:i + 1]
        S[:, r0:] = (np.abs(t.detJ) ** ((d - 1) / d))[:, None]
        self.S = S
        self.Jinv = np.linalg.inv(t.J)
        # operator quadrature (fixed by the method, see quadrature.py)
        self.xq, self.wq = simplex_rule(d, volume_points_per_dir(k))
        self.sq, self.wsq = simplex_rule(d - 1, facet_points_per_dir(k))
        self.ref_vals, self.ref_grads = B.dual_basis(d, k, self.xq)
        self.psi_q = B.psi(d, k, self.sq)  # [nqf][nf]
        self.psi_deg = np.array([B.facet_mode_degree(m) for m in B.facet_modes(d, k)])
        self.ref_face = []
        for i in range(d + 1):
            o, Em, _ = B.ref_facet_map(d, i)
            xh = o[None, :] + self.sq @ Em.T
            self.ref_face.append(B.dual_basis(d, k, xh)[0])  # [nqf][n][d]

    # ------------------------------------------------------------ helpers
    def local(self, x, elems):
        g = self.gdof[elems]
        return np.where(g >= 0, x[np.maximum(g, 0)], 0.0)

    def scatter(self, out, elems, vals):
        g = self.gdof[elems].ravel()
        v = vals.ravel()
        m = g >= 0
        np.add.at(out, g[m], v[m])

    def phys_vals(self, elems, ref_vals):
        """S J phi^ / det J for the given elements: [B][nq][n][d]."""
        t = self.topo
        J = t.J[elems]
        fac = self.S[elems] / t.detJ[elems][:, None]
        return np.einsum("bac,qic->bqia", J, ref_vals) * fac[:, None, :, None]

    def phys_grads(self, elems, ref_grads):
        """S J grad^phi^ J^{-1} / det J: [B][nq][n][d(comp)][d(deriv)]."""
        t = self.topo
        J = t.J[elems]
        Ji = self.Jinv[elems]
        fac = self.S[elems] / t.detJ[elems][:, None]
        g = J[:, None, None] @ ref_grads[None] @ Ji[:, None, None]
        return g * fac[:, None, :, None, None]

    def batches(self, n, size):
        for s in range(0, n, size):
            yield np.arange(s, min(n, s + size))

    def elem_batch_size(self):
        return max(1, int(2.0e7 // (len(self.wq) * self.n * self.dim * self.dim)))

    def facet_l(self, l):
        F = self.topo.n_facets
        if np.isscalar(l) or np.ndim(l) == 0:
            return np.full(F, int(l), dtype=np.int64)
        return np.asarray(l, dtype=np.int64)

    # --------------------------------------------------- interpolation
    def interpolate(self, field, nq1d=None, elems=None):
        """Canonical interpolant (the DoFs above applied to an analytic field),
        computed with a collapsed rule of nq1d points per direction.  With
        `elems`, only the DoFs of those elements (their facets' and their
        interior DoFs) are computed; every other DoF is zero."""
        t = self.topo
        d = self.dim
        nq1d = nq1d or (self.k + 8)
        x = np.zeros(self.n_dof)
        s, ws = simplex_rule(d - 1, nq1d)
        ps = B.psi(d, self.k, s)
        T = t.facet_elems[:, 0]
        i = t.facet_local[:, 0]
        facets = np.arange(t.n_facets)
        if elems is not None:
            fe = t.elem_facet[np.asarray(elems)].ravel()
            facets = np.unique(fe[fe >= 0])
        for f0 in range(0, len(facets), 4096):
            sl = facets[f0:f0 + 4096]
            Tb, ib = T[sl], i[sl]
            lv = np.array([[v for v in range(d + 1) if v != ii] for ii in ib])
            xv = np.take_along_axis(t.xyz[Tb], lv[:, :, None], 1)  # [B][d][d]
            pts = xv[:, None, 0, :] + np.einsum("bjc,qj->bqc",
                                                xv[:, 1:, :] - xv[:, :1, :], s)
            u = field(pts)
            nF = t.NF[Tb, ib] / t.NF_norm[Tb, ib][:, None]
            un = np.einsum("bqc,bc->bq", u, nF)
            vals = (un * ws[None, :]) @ ps  # [B][nf]
            x[(sl[:, None] * self.nf + np.arange(self.nf)[None, :])] = vals
        xq, wq = simplex_rule(d, nq1d)
        qm = B.interior_tests(d, self.k, xq)  # [nq][nint][d]
        off = t.n_facets * self.nf
        ebs = self.batches(t.n_elems, 4096) if elems is None else \
            (np.asarray(elems)[s0:s0 + 4096] for s0 in range(0, len(elems), 4096))
        for eb in ebs:
            pts = t.xyz[eb, 0][:, None, :] + np.einsum("bcj,qj->bqc", t.J[eb], xq)
            u = field(pts)
            uh = np.einsum("b,bjc,bqc->bqj", t.detJ[eb], self.Jinv[eb], u)
            vals = np.einsum("bqj,qmj,q->bm", uh, qm, wq)
            vals *= (np.abs(t.detJ[eb]) ** (-(d - 1) / d))[:, None]
            x[off + eb[:, None] * self.nint + np.arange(self.nint)[None, :]] = vals
        return x

    def evaluate(self, x, elems, ref_pts):
        """u at reference points of the given elements: [B][npts][d]."""
        vals, _ = B.dual_basis(self.dim, self.k, np.atleast_2d(ref_pts))
        phi = self.phys_vals(elems, vals)
        return np.einsum("bqid,bi->bqd", phi, self.local(x, elems))

    def physical_points(self, elems, ref_pts):
        t = self.topo
        return t.xyz[elems, 0][:, None, :] + np.einsum("bcj,qj->bqc", t.J[elems],
                                                          np.atleast_2d(ref_pts))
