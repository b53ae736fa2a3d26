"""Python front end of libhopu: a context object over torch device tensors
and torch.autograd.Functions for the substep chain (backward = the library's
hand-written adjoint)."""
import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import check, FP64, FP32_MFMA, BF16X2, BF16X3, TERM_ALL  # noqa: F401


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, n=None, dtype=torch.float64, what="vector"):
    """A tensor whose data pointer goes to the library: checked here, since
    the library cannot tell a short, host or mistyped buffer from a good one
    (n: the number of entries the call reads or writes)."""
    if not torch.is_tensor(t):
        raise TypeError(f"{what}: expected a torch tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what}: expected {n} entries, got {t.numel()}")
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{what}: expected a contiguous {dtype} tensor on the GPU")
    return t


def mfma_f64_rate(blocks_per_cu):
    """Sustained FP64 MFMA rate (TFLOP/s) of register-only 16x16x4 chains
    with blocks_per_cu blocks of four waves per CU (measurement helper)."""
    t = C.c_double()
    check(L.lib().hopu_mfma_f64_rate(int(blocks_per_cu), C.byref(t)), None)
    return t.value


class Hopu:
    """One velocity space on one mesh (see include/hopu.h)."""

    def __init__(self, dim, k, elem_vid, elem_xyz, device="cuda:0", stream=None):
        self.device = torch.device(device)
        vid = np.ascontiguousarray(elem_vid, dtype=np.int64)
        xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
        self.dim, self.k = dim, k
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = L.lib().hopu_create(C.byref(h), dim, k, vid.shape[0],
                                     vid.ctypes.data_as(C.c_void_p),
                                     xyz.ctypes.data_as(C.c_void_p),
                                     C.c_void_p(self.stream.cuda_stream))
        check(st, None)
        self.h = h
        nd, nf, nw = C.c_int64(), C.c_int64(), C.c_int64()
        nl, nfd, ni = C.c_int(), C.c_int(), C.c_int()
        check(L.lib().hopu_sizes(h, C.byref(nd), C.byref(nf), C.byref(nw), C.byref(nl),
                                 C.byref(nfd), C.byref(ni)), h)
        self.n_dof, self.n_facets, self.n_wall = nd.value, nf.value, nw.value
        self.n_loc, self.n_facet_dof, self.n_interior_dof = nl.value, nfd.value, ni.value
        self.n_elems = vid.shape[0]
        self._lfac = None

    def close(self):
        if getattr(self, "h", None):
            L.lib().hopu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros(self):
        return torch.zeros(self.n_dof, dtype=torch.float64, device=self.device)

    def set_upwind(self, l, l_per_facet=None):
        if l_per_facet is not None:
            _dev(l_per_facet, self.n_facets, torch.int8, "l_per_facet")
        self._lfac = l_per_facet  # the library keeps the pointer
        check(L.lib().hopu_set_upwind(self.h, int(l), _ptr(l_per_facet)), self.h)

    def jump_indicator(self, u):
        eta = torch.empty(self.n_facets, dtype=torch.float64, device=self.device)
        check(L.lib().hopu_jump_indicator(self.h, _ptr(_dev(u, self.n_dof)), _ptr(eta)), self.h)
        return eta

    def set_adaptive(self, every, thresholds=None, l_initial=-1):
        thr = None
        if thresholds is not None:
            thr = np.ascontiguousarray(thresholds, dtype=np.float64)
        check(L.lib().hopu_set_adaptive(self.h, int(every), 0 if thr is None else thr.size,
                                        None if thr is None else thr.ctypes.data_as(C.c_void_p),
                                        int(l_initial)), self.h)

    def adapt_upwind(self, u):
        check(L.lib().hopu_adapt_upwind(self.h, _ptr(_dev(u, self.n_dof))), self.h)

    def facet_orders(self):
        """The context's current per-facet orders (adaptive mode), int8."""
        out = torch.empty(self.n_facets, dtype=torch.int8, device=self.device)
        check(L.lib().hopu_get_facet_orders(self.h, _ptr(out)), self.h)
        return out

    def set_warm_start(self, carry):
        """carry: continue the PCG initial-guess extrapolation across
        substeps() calls (one trajectory advanced in several calls)."""
        check(L.lib().hopu_set_warm_start(self.h, int(bool(carry))), self.h)

    def set_solver(self, rtol=1e-13, max_it=500, check_every=4):
        check(L.lib().hopu_set_solver(self.h, float(rtol), int(max_it), int(check_every)), self.h)

    def apply(self, u, r=None, terms=TERM_ALL, prec=FP64):
        r = self.zeros() if r is None else r
        check(L.lib().hopu_convection_apply(self.h, _ptr(_dev(u, self.n_dof)), _ptr(_dev(r, self.n_dof)), terms, prec), self.h)
        return r

    def mass_apply(self, u, y=None):
        y = self.zeros() if y is None else y
        check(L.lib().hopu_mass_apply(self.h, _ptr(_dev(u, self.n_dof)), _ptr(_dev(y, self.n_dof))), self.h)
        return y

    def mass_solve(self, r, w=None, rtol=0.0, max_it=1000):
        w = self.zeros() if w is None else w
        its = C.c_int()
        check(L.lib().hopu_mass_solve(self.h, _ptr(_dev(r, self.n_dof)), _ptr(_dev(w, self.n_dof)), float(rtol), int(max_it),
                                      C.byref(its)), self.h)
        return w, its.value

    def project(self, ustar, out=None, rtol=1e-13, max_it=20000):
        """u_new = u* - u~ (projection step); returns (u_new, CG iterations)."""
        out = self.zeros() if out is None else out
        its = C.c_int()
        check(L.lib().hopu_project(self.h, _ptr(_dev(ustar, self.n_dof)), _ptr(_dev(out, self.n_dof)), float(rtol), int(max_it),
                                   C.byref(its)), self.h)
        return out, its.value

    def substeps(self, u, dt, n_steps, prec=FP64, diag=False):
        d = torch.zeros((n_steps + 1, 5), dtype=torch.float64, device=self.device) if diag else None
        check(L.lib().hopu_substeps(self.h, _ptr(_dev(u, self.n_dof)), float(dt), int(n_steps), prec, _ptr(d)), self.h)
        return d

    def vjp(self, u, mu, out=None, prec=FP64):
        out = self.zeros() if out is None else out
        check(L.lib().hopu_convection_vjp(self.h, _ptr(_dev(u, self.n_dof)), _ptr(_dev(mu, self.n_dof)), _ptr(_dev(out, self.n_dof)), prec), self.h)
        return out

    def substeps_vjp(self, u0, dt, n_steps, lam_N, ckpt_every=5, prec=FP64):
        nb = L.lib().hopu_substeps_vjp_workspace(self.h, int(n_steps), int(ckpt_every))
        if nb < 0:
            check(int(nb), self.h)
        ws = torch.empty(max(int(nb), 8), dtype=torch.uint8, device=self.device)
        lam0 = self.zeros()
        check(L.lib().hopu_substeps_vjp(self.h, _ptr(_dev(u0, self.n_dof)), float(dt), int(n_steps), int(ckpt_every),
                                        _ptr(_dev(lam_N, self.n_dof)), _ptr(lam0), prec, _ptr(ws), int(ws.numel())),
              self.h)
        return lam0

    def energy(self, u, out=None):
        """1/2 u.Mu as a 0-dim device tensor (no host synchronisation)."""
        out = torch.zeros((), dtype=torch.float64, device=self.device) if out is None else out
        check(L.lib().hopu_energy(self.h, _ptr(_dev(u, self.n_dof)), _ptr(_dev(out, 1, what="energy"))), self.h)
        return out

    def count_nonfinite(self, v):
        """Number of NaN / infinite entries of v."""
        n = C.c_int64()
        check(L.lib().hopu_count_nonfinite(self.h, _ptr(_dev(v, self.n_dof)), C.byref(n)), self.h)
        return n.value

    def diagnostics(self, u):
        e, dv, ds = C.c_double(), C.c_double(), C.c_double()
        check(L.lib().hopu_diagnostics(self.h, _ptr(_dev(u, self.n_dof)), C.byref(e), C.byref(dv), C.byref(ds)), self.h)
        return e.value, dv.value, ds.value

    def interp_points(self, n1d):
        d = self.dim
        nqf = n1d ** (d - 1)
        nqv = n1d ** d
        pf = torch.empty((self.n_facets, nqf, d), dtype=torch.float64, device=self.device)
        pv = torch.empty((self.n_elems, nqv, d), dtype=torch.float64, device=self.device)
        check(L.lib().hopu_interp_points(self.h, int(n1d), _ptr(pf), _ptr(pv)), self.h)
        return pf, pv

    def interpolate(self, field, n1d=None):
        """Coefficients of the canonical interpolant of `field` (callable on
        [..., d] tensors), sampled at the library's points."""
        n1d = n1d or (self.k + 2)
        pf, pv = self.interp_points(n1d)
        vf = _dev(field(pf).contiguous(), pf.numel(), what="field values at facet points")
        vv = _dev(field(pv).contiguous(), pv.numel(), what="field values at volume points")
        u = self.zeros()
        check(L.lib().hopu_interpolate(self.h, int(n1d), _ptr(vf), _ptr(vv), _ptr(u)), self.h)
        return u

    # ---- implicit Stokes step (hopu_stokes_*)
    def stokes_sizes(self):
        """(n_total, n_uhat, unknowns per element of S_T)."""
        nt, nh, nx = C.c_int64(), C.c_int64(), C.c_int()
        check(L.lib().hopu_stokes_sizes(self.h, C.byref(nt), C.byref(nh), C.byref(nx)), self.h)
        return nt.value, nh.value, nx.value

    def stokes_setup(self, nu, dt, fp32_precond=False):
        """Element Schur complements for (nu, dt); fp32_precond keeps S_T^-1 in FP32."""
        flags = L.HOPU_STOKES_FP32_PRECOND if fp32_precond else 0
        check(L.lib().hopu_stokes_setup(self.h, float(nu), float(dt), flags), self.h)

    def _stokes_vec(self, out):
        n = self.stokes_sizes()[0]
        return torch.zeros(n, dtype=torch.float64, device=self.device) if out is None else _dev(out, n)

    def stokes_apply(self, x, y=None):
        y = self._stokes_vec(y)
        check(L.lib().hopu_stokes_apply(self.h, _ptr(_dev(x, y.numel())), _ptr(y)), self.h)
        return y

    def stokes_precond(self, x, y=None):
        y = self._stokes_vec(y)
        check(L.lib().hopu_stokes_precond(self.h, _ptr(_dev(x, y.numel())), _ptr(y)), self.h)
        return y

    def stokes_step(self, un, with_convection=True, out=None, rtol=1e-12, max_it=2000, guess=False):
        """[u*; u^] of one implicit Stokes step from u^n; returns (x, iterations).
        guess: start the PCG from the contents of `out` (else from zero)."""
        if guess and out is None:
            raise ValueError("guess=True needs the initial guess in `out`")
        x = self._stokes_vec(out)
        flags = (L.HOPU_STOKES_CONVECTION if with_convection else 0) | (L.HOPU_STOKES_GUESS if guess else 0)
        its = C.c_int()
        check(L.lib().hopu_stokes_step(self.h, _ptr(_dev(un, self.n_dof)), flags, _ptr(x),
                                       float(rtol), int(max_it), C.byref(its)), self.h)
        return x, its.value

    PROF_KINDS = {"elem": 0, "mass": 1, "prec": 2, "modal": 3, "vjp": 4, "plain": 5,
                  "stokes_S": 6, "stokes_C": 7}

    def profile(self, enable, max_launches=200000):
        """enable: False/0 stops; True/1 times every launch of the main
        kernels; an int s > 1 times every s-th launch of each kind."""
        check(L.lib().hopu_profile_enable(self.h, int(enable), int(max_launches)), self.h)

    def profile_read(self, kind):
        n, ms = C.c_int64(), C.c_double()
        check(L.lib().hopu_profile_read(self.h, self.PROF_KINDS[kind], C.byref(n), C.byref(ms)), self.h)
        return n.value, ms.value

    def eval(self, u, ref_pts):
        ref = np.ascontiguousarray(ref_pts, dtype=np.float64)
        if ref.ndim != 2 or ref.shape[1] != self.dim:
            raise ValueError(f"ref_pts: expected shape [n_pts][{self.dim}], got {ref.shape}")
        out = torch.empty((self.n_elems, ref.shape[0], self.dim), dtype=torch.float64, device=self.device)
        check(L.lib().hopu_eval(self.h, _ptr(_dev(u, self.n_dof)), ref.shape[0],
                                ref.ctypes.data_as(C.c_void_p), _ptr(out)), self.h)
        return out


class SubstepChain(torch.autograd.Function):
    """u_N = S^n(u_0) with S(u) = u - dt M^-1 r(u); backward runs the
    library's checkpointed reverse pass."""

    @staticmethod
    def forward(ctx, u0, space, dt, n_steps, ckpt_every, prec):
        u = u0.detach().clone()
        space.substeps(u, dt, n_steps, prec)
        ctx.space, ctx.dt, ctx.n, ctx.ck, ctx.prec = space, dt, n_steps, ckpt_every, prec
        ctx.save_for_backward(u0.detach())
        return u

    @staticmethod
    def backward(ctx, g):
        (u0,) = ctx.saved_tensors
        lam0 = ctx.space.substeps_vjp(u0, ctx.dt, ctx.n, g.contiguous(), ctx.ck, ctx.prec)
        return lam0, None, None, None, None, None


class MassEnergy(torch.autograd.Function):
    """E(u) = 1/2 u.Mu (the library's energy) with gradient M u (the
    library's mass apply), scaled by the incoming gradient."""

    @staticmethod
    def forward(ctx, u, space):
        u = u.detach().contiguous()
        ctx.space = space
        ctx.save_for_backward(u)
        return space.energy(u)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        return g * ctx.space.mass_apply(u), None
