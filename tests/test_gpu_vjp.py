"""GPU adjoint: transpose-Jacobian parity with the oracle, identities,
checkpointing, central finite differences on the 3D periodic curl-field
adjoint workload, and the autograd path."""
import numpy as np
import pytest
import torch

import synth
from synth.configs import fd_directions
from oracle import operator as O
from gpu_util import case, gpu_space, dev, host, rel_dual, rel_primal, check_dual, check_mixed

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,n,k", [(1, (6, 5), 2), (4, (3, 3, 3), 2), (2, (4, 3, 3), 3), (3, (3, 5, 3), 4),
                                     (3, (3, 3, 4), 5)])
def test_vjp_matches_oracle(cfg, n, k):
    mesh, sp, x, c = case(cfg, n, k, noise=1e-2)
    mu = np.random.default_rng(11).standard_normal(sp.n_dof)
    h = gpu_space(mesh, k)
    for l in (-1, k - 1):
        h.set_upwind(l)
        g = host(h.vjp(dev(x), dev(mu)))
        ref = O.vjp(sp, x, mu, l)
        check_dual(sp, g, ref, 1e-12, f"vjp cfg={cfg} k={k} l={l}")


@pytest.mark.parametrize("cfg,n,k", [(1, (6, 5), 2), (2, (4, 3, 3), 3), (3, (3, 3, 4), 5)])
def test_vjp_fp32_matches_oracle(cfg, n, k):
    """FP32-MFMA adjoint against the FP64 oracle, with the FP32-MFMA bound of
    the forward apply (the same contractions; modal and dual transforms in
    FP64), up to k = 5 on the walled, graded, jittered mesh."""
    mesh, sp, x, c = case(cfg, n, k, noise=1e-2)
    mu = np.random.default_rng(11).standard_normal(sp.n_dof)
    h = gpu_space(mesh, k)
    h.set_upwind(k - 1)
    g = host(h.vjp(dev(x), dev(mu), prec=1))
    ref = O.vjp(sp, x, mu, k - 1)
    # 1e-6 in 3D; the 2D k = 2 case carries the cancellation of the forward
    # apply (volume and central parts each 8 times the sum): 3e-6
    check_mixed(sp, g, ref, 3e-6 if cfg == 1 else 1e-6, f"vjp fp32 cfg={cfg} k={k}")


def test_vjp_at_zero_normal_velocity():
    """The shear field (p(y), 0, q(y)) on the walled, graded, jittered mesh
    has u.n = 0 on every facet whose normal is along y (and no jumps): the
    transpose Jacobian there (reading sgn(0) = 0) matches the oracle."""
    from synth import fields
    mesh, sp, _, c = case(3, (3, 5, 3), 3, noise=0.0)
    x = sp.interpolate(fields.shear_field([0.2, 1.0, -0.8], [0.1, -0.5, 0.3]))
    mu = np.random.default_rng(12).standard_normal(sp.n_dof)
    h = gpu_space(mesh, 3)
    for l in (-1, 2):
        h.set_upwind(l)
        g = host(h.vjp(dev(x), dev(mu)))
        check_dual(sp, g, O.vjp(sp, x, mu, l), 1e-12, f"vjp shear l={l}")


@pytest.mark.parametrize("cfg,n,k", [(2, (4, 3, 3), 3), (3, (3, 5, 3), 4), (3, (3, 3, 4), 5)])
@pytest.mark.parametrize("prec", [2, 3])
def test_vjp_bf16_split_matches_oracle(cfg, n, k, prec):
    """Split-BF16 transpose Jacobian (the forward kernel's split contractions
    plus split copies of its two volume tables) against the FP64 oracle:
    hi/mid/lo carries the FP32 operands exactly and is held to 1e-6; hi/lo
    to its apply bound 3e-3."""
    mesh, sp, x, c = case(cfg, n, k, noise=1e-2)
    mu = np.random.default_rng(11).standard_normal(sp.n_dof)
    h = gpu_space(mesh, k)
    h.set_upwind(k - 1)
    ref = O.vjp(sp, x, mu, k - 1)
    g = host(h.vjp(dev(x), dev(mu), prec=prec))
    check_mixed(sp, g, ref, 1e-6 if prec == 3 else 3e-3, f"vjp bf16x{prec} cfg={cfg} k={k}")


def test_chain_vjp_bf16x3():
    """The checkpointed reverse chain with hi/mid/lo contractions on the
    walled, graded mesh at k = 4 against the oracle's chain adjoint."""
    mesh, sp, x, c = case(3, (3, 4, 3), 4, noise=1e-2)
    h = gpu_space(mesh, 4)
    h.set_upwind(3)
    h.set_solver(rtol=1e-13, max_it=2000)
    dt, n = 1e-3, 3
    xN = O.substeps(sp, x, dt, n, 3)
    lamN = O.mass_apply(sp, xN)
    ref = O.chain_vjp(sp, x, dt, n, 3, lamN)
    g = host(h.substeps_vjp(dev(x), dt, n, dev(lamN), ckpt_every=2, prec=3))
    check_mixed(sp, g, ref, 1e-6, "chain vjp bf16x3 (k = 4)")


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)])
def test_vjp_homogeneity_and_fd(prec, tol):
    """J_r(u) u = 2 r(u) (r is positively homogeneous of degree 2), and the
    dot-product test <J_r delta, mu> = <delta, J_r^T mu> with central FD."""
    mesh, sp, x, c = case(2, (4, 4, 3), 3, noise=1e-2)
    h = gpu_space(mesh, 3)
    h.set_upwind(2)
    rng = np.random.default_rng(5)
    mu = dev(rng.standard_normal(sp.n_dof))
    u = dev(x)
    g = h.vjp(u, mu, prec=prec)
    r = h.apply(u, prec=prec)
    lhs, rhs = float(torch.dot(g, u)), 2 * float(torch.dot(mu, r))
    assert abs(lhs - rhs) <= tol * abs(rhs)
    if prec == 0:
        hh = 1e-6
        for _ in range(3):
            d = dev(rng.standard_normal(sp.n_dof))
            fd = float(torch.dot(mu, h.apply(u + hh * d) - h.apply(u - hh * d))) / (2 * hh)
            assert abs(fd - float(torch.dot(d, g))) <= 1e-7 * abs(fd)


def test_chain_vjp_matches_oracle():
    mesh, sp, x, c = case(1, (8, 8), 2, noise=1e-2)
    h = gpu_space(mesh, 2)
    h.set_upwind(1)
    h.set_solver(rtol=1e-13, max_it=2000)
    dt, n = 1e-2, 4
    xN = O.substeps(sp, x, dt, n, 1)
    lamN = O.mass_apply(sp, xN)
    ref = O.chain_vjp(sp, x, dt, n, 1, lamN)
    g = host(h.substeps_vjp(dev(x), dt, n, dev(lamN), ckpt_every=2))
    assert rel_dual(sp, g, ref) <= 1e-11
    # FP32-MFMA reverse chain: lam_0 = lam_N + O(dt) terms, so its error
    # relative to lam_0 is below that of one vjp
    gp = host(h.substeps_vjp(dev(x), dt, n, dev(lamN), ckpt_every=2, prec=1))
    check_mixed(sp, gp, ref, 3e-6, "chain vjp fp32 (2D k = 2)")


def test_checkpointing_is_bitwise():
    mesh, sp, x, c = case(2, (4, 3, 3), 3, noise=1e-2)
    h = gpu_space(mesh, 3)
    h.set_upwind(2)
    u0 = dev(x)
    lam = dev(np.random.default_rng(1).standard_normal(sp.n_dof))
    a = host(h.substeps_vjp(u0, 1e-3, 7, lam, ckpt_every=1))
    b = host(h.substeps_vjp(u0, 1e-3, 7, lam, ckpt_every=3))
    cc = host(h.substeps_vjp(u0, 1e-3, 7, lam, ckpt_every=7))
    assert np.array_equal(a, b) and np.array_equal(a, cc)


def test_adjoint_fd_curl_workload():
    """3D periodic [0,2pi]^3, 24^3 x 6 tets, k = 3, divergence-free random
    Fourier curl field (|n| <= 4, RMS 1), loss = kinetic energy after 20
    substeps at dt = 1e-3 (l = 2), checkpoint every 5; central FD with
    h = 1e-6 on 32 seeded directions scaled to ||delta||_M = ||u0||_M."""
    from paper_2408_06698_amd.hopu import Hopu, SubstepChain, MassEnergy
    mesh, field, cfg = synth.make_config(4)
    h = Hopu(3, cfg["k"], mesh.elem_vid, mesh.elem_xyz)
    h.set_upwind(cfg["l"])
    # the FD quotient divides solver noise in the states by 2h = 2e-6:
    # solve the mass systems to 1e-14 (preconditioned residual)
    h.set_solver(rtol=1e-14, max_it=4000)
    u0 = h.interpolate(field, n1d=cfg["k"] + 3)
    dt, n, ck = cfg["dt"], cfg["steps"], cfg["ckpt_every"]

    def final(u):
        v = u.clone()
        h.substeps(v, dt, n)
        return v

    uN = u0.clone()
    h.substeps(uN, dt, n)
    lam0 = h.substeps_vjp(u0, dt, n, h.mass_apply(uN), ckpt_every=ck)
    # the autograd path gives the same gradient
    x = u0.clone().requires_grad_(True)
    L = MassEnergy.apply(SubstepChain.apply(x, h, dt, n, ck, 0), h)
    L.backward()
    assert torch.equal(x.grad, lam0)
    nrm0 = float(torch.sqrt(torch.dot(u0, h.mass_apply(u0))))
    dirs = fd_directions(4, cfg["fd_dirs"], h.n_dof)
    gnorm = float(torch.sqrt(torch.dot(lam0, h.mass_solve(lam0.clone(), rtol=1e-14, max_it=4000)[0])))

    def fd_errors(hh):
        errs, nerrs = [], []
        for i in range(cfg["fd_dirs"]):
            d = dev(dirs[i])
            d *= nrm0 / float(torch.sqrt(torch.dot(d, h.mass_apply(d))))
            up, um = final(u0 + hh * d), final(u0 - hh * d)
            # (L+ - L-)/2h written as 1/2 (u+ - u-)^T M (u+ + u-)/2h: a random
            # direction is nearly M-orthogonal to the gradient, and subtracting
            # the two O(1e2) losses would cancel most significant digits
            fd = 0.5 * float(torch.dot(up - um, h.mass_apply(up + um))) / (2 * hh)
            ad = float(torch.dot(lam0, d))
            errs.append(abs(fd - ad) / abs(fd))
            nerrs.append(abs(fd - ad) / (gnorm * nrm0))
        return np.array(errs), np.array(nerrs)

    # h = 1e-6 (the workload's step): the per-direction ratio |fd-ad|/|fd|
    # is rounding noise magnified by the direction's near-orthogonality to
    # the gradient (cos 3e-4 .. 1e-2); the oracle's own h-sweep on this
    # recipe (4^3 x 6 tets, exact solves) shows the noise growing as 1/h
    # below h = 1e-5 (2e-8 at 1e-6, 1e-7 at 1e-7, 4e-6 at 1e-8) and the
    # truncation error growing as h^2 above it, with the minimum (1e-9 ..
    # 1e-10) at h = 1e-5.  So: every direction at h = 1e-5 within 1e-7;
    # at h = 1e-6 the gradient-normalised error and the median.
    errs, nerrs = fd_errors(cfg["fd_h"])
    errs5, nerrs5 = fd_errors(1e-5)
    print(f"adjoint FD, {cfg['fd_dirs']} directions, h = 1e-6: |fd-ad|/|fd| " +
          " ".join(f"{e:.1e}" for e in errs))
    print(f"adjoint FD, h = 1e-6: max {errs.max():.2e} median {np.median(errs):.2e}; "
          f"|fd-ad|/(|grad L| |delta|) max {nerrs.max():.2e}")
    print(f"adjoint FD, h = 1e-5: |fd-ad|/|fd| max {errs5.max():.2e} median {np.median(errs5):.2e}")
    assert errs5.max() <= 1e-7
    assert nerrs.max() <= 1e-10
    assert np.median(errs) <= 1e-7
