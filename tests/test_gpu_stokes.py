"""GPU parity of the implicit Stokes step (paper section 2.2, spaces and
forms; section 2.3, eq. (MCS_step1), static condensation, element-wise BDDC)
against the oracle, through the C ABI: the condensed operator S x, the
preconditioner C^-1 x, and the step's (u*, u^) with and without the
convection term.  FP64 throughout; entry-wise comparison, relative to the
largest entry of each block (velocity, u^)."""
import numpy as np
import pytest
import torch

import synth
from oracle import operator as O
from oracle import stokes as OST
from oracle.space import Space
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _case(d, k, n, walls, jitter=0.1):
    per = tuple(a != 1 for a in range(d)) if walls else (True,) * d
    m = synth.kuhn_mesh(d, (n,) * d, periodic=per, jitter=jitter, jitter_seed=9 if jitter else None)
    return m, Space(m.elem_vid, m.elem_xyz, k)


def _gpu(m, k):
    from paper_2408_06698_amd.hopu import Hopu
    return Hopu(m.dim, k, m.elem_vid, m.elem_xyz)


def _blockerr(sp, v, ref):
    nd = sp.n_dof
    out = []
    for sl in (slice(0, nd), slice(nd, len(ref))):
        den = np.abs(ref[sl]).max()
        out.append(float(np.abs(v[sl] - ref[sl]).max() / den))
    return max(out)


# The two sides condense sigma and gamma through different bases (the
# oracle: reference-coordinate monomials and a null-space reduction; the
# library: an orthonormal Dubiner basis with multipliers), so their
# rounding differs by the conditioning of the element blocks, which grows
# with k: the bounds below (entry-wise, relative to each block's largest
# entry) follow the CPU emulation of the set-up against the oracle (S x:
# 1e-14, 6e-13, 2.4e-11, 2.9e-9 at 2D k = 1..4; 1.3e-13, 6.2e-12, 3.4e-10 at
# 3D k = 1..3, 1.06e-7 at 3D k = 4, where per element the gap is 1e-9 to
# 6e-9 and S x cancels); C^-1 adds the conditioning of S_T (3D k = 4:
# 9.7e-9).  Against that emulation
# (same formulas, LAPACK in numpy) the GPU's S x agrees to rounding
# (EMU_TOL): the kernel's own arithmetic is pinned tighter than the two
# condensation routes agree.
TOL_S = {1: 1e-12, 2: 1e-11, 3: 1e-9, 4: 1e-8, (3, 4): 3e-7}
TOL_C = {1: 1e-10, 2: 1e-10, 3: 5e-9, 4: 1e-7}
EMU_TOL = 1e-12
TOL_STEP = {1: 1e-10, 2: 1e-10, 3: 1e-9}

def _emulated_S(m, sp, k, nu, dt, schur):
    """S assembled from the CPU emulation of the set-up kernel."""
    import scipy.sparse as sps
    from tests.test_stokes_setup_math import emulate_ST, _table, _frames
    loc = schur[2]
    tabs = [_table(m.dim, k, w) for w in range(20, 26)]
    geo = _frames(m)
    rows, cols, vals = [], [], []
    for T in range(sp.topo.n_elems):
        Se = emulate_ST(m.dim, k, geo[T], nu, dt, tabs)
        g = loc[T]
        rr = np.broadcast_to(g[:, None], Se.shape)
        cc = np.broadcast_to(g[None, :], Se.shape)
        keep = (rr >= 0) & (cc >= 0)
        rows.append(rr[keep]); cols.append(cc[keep]); vals.append(Se[keep])
    return sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=schur[0].shape).tocsr()


CASES = [(2, 1, 4, False), (2, 2, 4, True), (2, 3, 3, False), (2, 4, 3, True),
         (3, 1, 3, False), (3, 2, 3, True), (3, 3, 3, False), (3, 4, 3, False)]


@pytest.mark.parametrize("d,k,n,walls", CASES)
def test_stokes_operator_and_preconditioner(d, k, n, walls):
    print(f"stokes S/C^-1 d={d} k={k} n={n} walls={walls}", flush=True)
    m, sp = _case(d, k, n, walls)
    nu, dt = 0.03, 0.01
    schur = OST.schur_system(sp, nu, dt)
    g = _gpu(m, k)
    nt, nh, nx = g.stokes_sizes()
    assert nt == schur[0].shape[0] and nh == OST.n_uhat(sp)
    g.stokes_setup(nu, dt)
    rng = np.random.default_rng(100 + 10 * d + k)
    x = rng.standard_normal(nt)
    y = host(g.stokes_apply(dev(x)))
    ref = schur[0] @ x
    print(f"  S x: {_blockerr(sp, y, ref):.2e}", flush=True)
    assert _blockerr(sp, y, ref) <= TOL_S.get((d, k), TOL_S[k])
    yemu = _emulated_S(m, sp, k, nu, dt, schur) @ x
    print(f"  S x against the set-up emulation: {_blockerr(sp, y, yemu):.2e}", flush=True)
    assert _blockerr(sp, y, yemu) <= EMU_TOL
    z = host(g.stokes_precond(dev(x)))
    zref = OST.bddc_apply(sp, schur, x)
    print(f"  C^-1 x: {_blockerr(sp, z, zref):.2e}", flush=True)
    assert _blockerr(sp, z, zref) <= TOL_C[k]
    # S is symmetric: x . S y = y . S x for the GPU operator too
    y2 = rng.standard_normal(nt)
    a = x @ host(g.stokes_apply(dev(y2)))
    b = y2 @ y
    assert abs(a - b) <= 1e-12 * abs(a) * 10


@pytest.mark.parametrize("d,k,n,walls,conv", [(2, 2, 4, True, True), (2, 3, 3, False, True),
                                             (3, 1, 3, False, True), (3, 2, 3, True, True),
                                             (3, 2, 3, False, False)])
def test_stokes_step_matches_direct_solve(d, k, n, walls, conv):
    print(f"stokes step d={d} k={k} n={n} walls={walls} conv={conv}", flush=True)
    m, sp = _case(d, k, n, walls)
    f = (lambda x: np.stack([np.sin(np.pi * x[..., 1])] + [0.0 * x[..., 0]] * (d - 1), -1)) if walls else \
        (synth.taylor_green_2d() if d == 2 else synth.taylor_green_3d())
    un = sp.interpolate(f) + 1e-2 * np.random.default_rng(7).standard_normal(sp.n_dof)
    nu, dt = 0.05, 0.02
    r = O.residual(sp, un, -1) if conv else None
    us, uh, _, _, _ = OST.step1(sp, un, nu, dt, r)
    g = _gpu(m, k)
    g.set_upwind(-1)
    g.stokes_setup(nu, dt)
    x, its = g.stokes_step(dev(un), with_convection=conv, rtol=1e-13)
    xh = host(x)
    ref = np.concatenate([us, uh])
    print(f"  step: {_blockerr(sp, xh, ref):.2e} after {its} iterations", flush=True)
    assert _blockerr(sp, xh, ref) <= TOL_STEP[k], its
    assert its < 300


def test_stokes_errors_and_setup_reuse():
    print("stokes errors", flush=True)
    from paper_2408_06698_amd._lib import HopuError, HOPU_EINVAL, HOPU_EUNSUPPORTED
    m, sp = _case(2, 2, 3, False)
    g = _gpu(m, 2)
    nt = g.stokes_sizes()[0]
    x = torch.zeros(nt, dtype=torch.float64, device="cuda:0")
    with pytest.raises(HopuError) as e:
        g.stokes_apply(x)
    assert e.value.status == HOPU_EINVAL
    with pytest.raises(HopuError) as e:
        g.stokes_setup(-1.0, 0.1)
    assert e.value.status == HOPU_EINVAL
    # a second set-up with other nu, dt replaces the element matrices
    rng = np.random.default_rng(3)
    xv = rng.standard_normal(nt)
    for nu, dt in ((0.1, 0.05), (0.01, 0.2)):
        g.stokes_setup(nu, dt)
        y = host(g.stokes_apply(dev(xv)))
        ref = OST.schur_system(sp, nu, dt)[0] @ xv
        assert _blockerr(sp, y, ref) <= 1e-11
    m3 = synth.kuhn_mesh(3, (3, 3, 3), periodic=(True,) * 3)
    g4 = _gpu(m3, 5)
    with pytest.raises(HopuError) as e:
        g4.stokes_setup(0.1, 0.1)
    assert e.value.status == HOPU_EUNSUPPORTED


def test_stokes_step_decay_factor_at_size():
    """The 32^3 x 6 Taylor-Green mesh (k = 3) at the bench's nu and dt: the
    Stokes part alone maps the interpolated mode to (1 + 3 nu dt)^-1 times
    itself up to the discretisation error (a property that holds at any
    size; the oracle cannot run this mesh)."""
    print("stokes step 32^3 k=3", flush=True)
    L = (2 * np.pi,) * 3
    m = synth.kuhn_mesh(3, (32, 32, 32), periodic=(True,) * 3, lengths=L)
    g = _gpu(m, 3)
    nu, dt = 0.05, 0.05
    g.stokes_setup(nu, dt)
    tg = synth.taylor_green_3d()
    un = g.interpolate(tg)
    x, its = g.stokes_step(un, with_convection=False, rtol=1e-10)
    u = x[:g.n_dof]
    e = u - un / (1 + 3 * nu * dt)
    Me = g.mass_apply(e.contiguous())
    Mu = g.mass_apply(un)
    rel = float(torch.sqrt((e * Me).sum() / (un * Mu).sum()))
    print(f"  iterations {its}, relative M-norm error {rel:.3e}", flush=True)
    assert rel <= 1e-4


def test_stokes_step_initial_guess():
    """HOPU_STOKES_GUESS: the PCG from a guess reaches the same solution as
    from zero (to the stopping rule), in fewer iterations from a nearby
    solution, and from the solution itself in at most one."""
    print("stokes step with a guess", flush=True)
    m, sp = _case(3, 2, 3, True)
    f = lambda x: np.stack([np.sin(np.pi * x[..., 1]), 0.0 * x[..., 0], 0.0 * x[..., 0]], -1)
    un = sp.interpolate(f)
    g = _gpu(m, 2)
    g.stokes_setup(0.05, 0.02)
    u = dev(un)
    x0, its0 = g.stokes_step(u, rtol=1e-12)
    ref = host(x0)
    # a good guess: the solution from a nearby state (the previous step of a
    # time loop); [u^n; 0] is not one (u^ = 0 contradicts u's tangential trace)
    near = u + dev(1e-3 * np.random.default_rng(1).standard_normal(g.n_dof))
    xg, _ = g.stokes_step(near, rtol=1e-12)
    x1, its1 = g.stokes_step(u, out=xg, rtol=1e-12, guess=True)
    assert _blockerr(sp, host(x1), ref) <= 1e-10
    assert its1 < its0, (its1, its0)
    x2, its2 = g.stokes_step(u, out=x0.clone(), rtol=1e-12, guess=True)
    assert its2 <= 1 and _blockerr(sp, host(x2), ref) <= 1e-12


@pytest.mark.parametrize("d,k,n,walls", [(2, 2, 4, True), (3, 2, 3, True), (3, 3, 3, False)])
def test_stokes_fp32_preconditioner(d, k, n, walls):
    """HOPU_STOKES_FP32_PRECOND: S_T^-1 kept in FP32 (element products in
    FP64 arithmetic).  C^-1 x then carries the FP32 rounding of S_T^-1's
    entries (2^-24 relative, summed over nx terms); S, the vectors and the
    inner products stay FP64, so the step meets the FP64 tolerance."""
    print(f"stokes fp32 preconditioner d={d} k={k} n={n} walls={walls}", flush=True)
    m, sp = _case(d, k, n, walls)
    nu, dt = 0.05, 0.02
    schur = OST.schur_system(sp, nu, dt)
    g = _gpu(m, k)
    g.stokes_setup(nu, dt, fp32_precond=True)
    nt = g.stokes_sizes()[0]
    x = np.random.default_rng(5).standard_normal(nt)
    z = host(g.stokes_precond(dev(x)))
    zref = OST.bddc_apply(sp, schur, x)
    ez = _blockerr(sp, z, zref)
    print(f"  C^-1 x (FP32 S_T^-1): {ez:.2e}", flush=True)
    assert ez <= 2e-5
    f = (lambda xx: np.stack([np.sin(np.pi * xx[..., 1])] + [0.0 * xx[..., 0]] * (d - 1), -1)) if walls else \
        (synth.taylor_green_2d() if d == 2 else synth.taylor_green_3d())
    un = sp.interpolate(f) + 1e-2 * np.random.default_rng(7).standard_normal(sp.n_dof)
    r = O.residual(sp, un, -1)
    us, uh, _, _, _ = OST.step1(sp, un, nu, dt, r)
    g.set_upwind(-1)
    xs, its = g.stokes_step(dev(un), rtol=1e-13)
    e = _blockerr(sp, host(xs), np.concatenate([us, uh]))
    print(f"  step: {e:.2e} after {its} iterations", flush=True)
    assert e <= TOL_STEP[k]


def test_stokes_operator_graded_wall_mesh():
    """S and C^-1 on wall cells of aspect ratio 167 (y nodes 0, 0.002, 0.01,
    0.05, 0.2, 0.5, 1 under 3 x 3 periodic cubes, 5% jitter), k = 2, against
    the oracle and the set-up emulation.  (The PCG on S with the element-wise
    BDDC needs thousands of iterations on such flat tetrahedra, as the mass
    PCG does; the step is not run here.)"""
    print("stokes S/C^-1 graded wall mesh", flush=True)
    y = np.array([0.0, 0.002, 0.01, 0.05, 0.2, 0.5, 1.0])
    m = synth.kuhn_mesh(3, (3, 6, 3), periodic=(True, False, True), nodes=[None, y, None], jitter=0.05,
                        jitter_seed=5)
    sp = Space(m.elem_vid, m.elem_xyz, 2)
    nu, dt = 1e-3, 1e-3
    schur = OST.schur_system(sp, nu, dt)
    g = _gpu(m, 2)
    g.stokes_setup(nu, dt)
    nt = g.stokes_sizes()[0]
    x = np.random.default_rng(8).standard_normal(nt)
    y1 = host(g.stokes_apply(dev(x)))
    e_or = _blockerr(sp, y1, schur[0] @ x)
    e_emu = _blockerr(sp, y1, _emulated_S(m, sp, 2, nu, dt, schur) @ x)
    z = host(g.stokes_precond(dev(x)))
    e_c = _blockerr(sp, z, OST.bddc_apply(sp, schur, x))
    print(f"  S x: {e_or:.2e} (emulation {e_emu:.2e}), C^-1 x: {e_c:.2e}", flush=True)
    assert e_or <= 1e-10 and e_emu <= EMU_TOL and e_c <= 1e-8


def test_stokes_setup_refused_allocation_then_retry():
    """A refused allocation in the first set-up returns HOPU_ENOMEM and
    leaves the context usable: the next set-up allocates and works."""
    import os
    from paper_2408_06698_amd._lib import HopuError, HOPU_ENOMEM
    print("stokes set-up: refused allocation, then retry", flush=True)
    m, sp = _case(2, 2, 3, False)
    g = _gpu(m, 2)
    os.environ["HOPU_TEST_FAIL_ALLOC"] = "1"
    try:
        with pytest.raises(HopuError) as e:
            g.stokes_setup(0.1, 0.05)
        assert e.value.status == HOPU_ENOMEM
    finally:
        del os.environ["HOPU_TEST_FAIL_ALLOC"]
    g.stokes_setup(0.1, 0.05)
    x = np.random.default_rng(2).standard_normal(g.stokes_sizes()[0])
    y = host(g.stokes_apply(dev(x)))
    assert _blockerr(sp, y, OST.schur_system(sp, 0.1, 0.05)[0] @ x) <= 1e-11


def test_stokes_full_size_sampled_columns():
    """At the bench's size and parameters (32^3 x 6 Taylor-Green mesh, k = 3,
    nu = 1/1600, dt = 5e-4): columns of S and C^-1 at sampled unknowns (a
    velocity facet DoF, a u^ unknown and an interior DoF of seeded elements)
    against the oracle's element blocks of the elements that hold them.  The
    GPU applies S and C^-1 to unit vectors; every other entry must be zero."""
    print("stokes full-size sampled columns", flush=True)
    mesh, field, cfg = synth.make_config(2)
    sp = Space(mesh.elem_vid, mesh.elem_xyz, cfg["k"])
    nu, dt = 1.0 / 1600.0, cfg["dt"]
    g = _gpu(mesh, cfg["k"])
    g.stokes_setup(nu, dt)
    nt = g.stokes_sizes()[0]
    hg = OST.uhat_gdof(sp)
    loc = np.concatenate([sp.gdof, np.where(hg >= 0, sp.n_dof + hg, -1)], 1)
    nh = hg.shape[1]
    rng = np.random.default_rng(2408)
    elems = rng.choice(sp.topo.n_elems, 2, replace=False)
    cache = {}

    def st(T):
        if T not in cache:
            cache[T] = OST._schur_block(sp, OST.element_blocks(sp, T, nu), T, dt, nh)
        return cache[T]

    for T in elems:
        for li in (1, sp.n + 2, (sp.dim + 1) * sp.nf + 3):  # facet DoF, u^, interior DoF
            gi = int(loc[T, li])
            owners = np.nonzero((loc == gi).any(1))[0]
            ref_s = np.zeros(nt)
            ref_c = np.zeros(nt)
            for T2 in owners:
                S_T = st(T2)
                keep = loc[T2] >= 0
                l2 = int(np.nonzero(loc[T2] == gi)[0][0])
                ref_s[loc[T2][keep]] += S_T[keep, l2]
                w = np.where(np.arange(loc.shape[1]) < (sp.dim + 1) * sp.nf, 0.5, 1.0)
                w[sp.n:] = 0.5
                e = np.zeros(keep.sum())
                e[np.nonzero(keep)[0].tolist().index(l2)] = w[l2]
                z = np.linalg.solve(S_T[np.ix_(keep, keep)], e)
                ref_c[loc[T2][keep]] += w[keep] * z
            x = np.zeros(nt)
            x[gi] = 1.0
            ys = host(g.stokes_apply(dev(x)))
            yc = host(g.stokes_precond(dev(x)))
            es = np.abs(ys - ref_s).max() / np.abs(ref_s).max()
            ec = np.abs(yc - ref_c).max() / np.abs(ref_c).max()
            print(f"  element {T} local {li} ({len(owners)} owners): S {es:.2e}, C^-1 {ec:.2e}", flush=True)
            assert es <= 1e-9 and ec <= 1e-9
