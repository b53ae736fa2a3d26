"""GPU parity of the mass solve (PCG with the element-wise preconditioner),
explicit substeps and diagnostics against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import operator as O
from gpu_util import case, gpu_space, dev, host, rel_dual, rel_primal, check_primal

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,n,k", [(1, (16, 16), 2), (2, (4, 3, 3), 3), (3, (3, 5, 3), 4), (3, (3, 3, 4), 5)])
def test_mass_solve(cfg, n, k):
    mesh, sp, x, c = case(cfg, n, k, noise=1e-3)
    h = gpu_space(mesh, k)
    r = O.residual(sp, x, k - 1)
    w, its = h.mass_solve(dev(r), rtol=1e-13, max_it=2000)
    w = host(w)
    ref = O.mass_solve(sp, r)
    e = rel_primal(sp, w, ref)
    print(f"mass solve cfg={cfg} k={k} iters={its} rel={e:.2e}")
    assert e <= 1e-12


def test_mass_solve_zero_rhs():
    # the initial residual already meets rtol: no iteration, no update
    mesh, sp, x, c = case(2, (4, 3, 3), 3, noise=1e-3)
    h = gpu_space(mesh, 3)
    h.mass_solve(dev(O.residual(sp, x, 2)), rtol=1e-13)  # leaves solver scalars behind
    w, its = h.mass_solve(dev(np.zeros(sp.n_dof)), rtol=1e-13)
    assert its == 0 and not host(w).any()


def test_mass_solve_warm_start_and_noconv():
    mesh, sp, x, c = case(2, (4, 3, 3), 3, noise=1e-3)
    h = gpu_space(mesh, 3)
    r = O.residual(sp, x, 2)
    ref = O.mass_solve(sp, r)
    w0 = dev(ref * (1 + 1e-6))
    w, its = h.mass_solve(dev(r), w=w0, rtol=1e-13)
    assert rel_primal(sp, host(w), ref) <= 1e-12
    _, its_cold = h.mass_solve(dev(r), rtol=1e-13)
    assert its < its_cold
    from paper_2408_06698_amd._lib import HopuError
    with pytest.raises(HopuError) as ei:
        h.mass_solve(dev(r), rtol=1e-13, max_it=1)
    assert ei.value.status == -5


@pytest.mark.parametrize("cfg,n,k,steps,dt", [(1, (16, 16), 2, 10, 1e-3), (2, (4, 3, 3), 3, 4, 5e-4),
                                              (3, (3, 5, 3), 4, 3, 1e-4)])
def test_substeps_chain(cfg, n, k, steps, dt):
    """The workload-1 chain (10 substeps at dt = 1e-3, l = 1) and shorter
    3D chains, against the oracle's substeps with an exact mass solve."""
    mesh, sp, x, c = case(cfg, n, k)
    l = c["l"] if k == c["k"] else k - 1
    h = gpu_space(mesh, k)
    h.set_upwind(l)
    h.set_solver(rtol=1e-13, max_it=2000)
    u = dev(x)
    diag = h.substeps(u, dt, steps, diag=True)
    xs = O.substeps(sp, x, dt, steps, l, keep=True)
    ug = host(u)
    check_primal(sp, ug, xs[-1], 1e-12, f"substeps cfg={cfg} k={k}")
    d = host(diag)
    # diagnostics of the states the test holds exactly (the input and the
    # GPU's final state) against the oracle's on the same state: energy,
    # ||div u||_L2 and dissipation to 1e-12
    # (||div u|| of a nearly divergence-free state is a small difference of
    # O(|grad u|) terms: its rounding floor is ~1e-15 ||u||, so the bound
    # is 1e-12 relative plus 1e-14 ||u||_L2)
    for s, xv in ((0, x), (steps, ug)):
        E, dv, D = O.energy(sp, xv), O.divergence_l2(sp, xv), O.dissipation(sp, xv, l)
        print(f"diag state {s}: E {d[s, 0]:.6e}/{E:.6e} div {d[s, 1]:.6e}/{dv:.6e} diss {d[s, 2]:.6e}/{D:.6e}")
        assert abs(d[s, 0] - E) <= 1e-12 * E
        assert abs(d[s, 1] - dv) <= 1e-12 * dv + 1e-14 * np.sqrt(2 * E)
        assert abs(d[s, 2] - D) <= 1e-12 * D
    # the middle state (held only through the oracle's chain, 1e-12 away)
    s = steps // 2
    E = O.energy(sp, xs[s])
    assert abs(d[s, 0] - E) <= 1e-12 * E
    assert abs(d[s, 1] - O.divergence_l2(sp, xs[s])) <= 1e-11 * O.divergence_l2(sp, xs[s]) + 1e-13 * np.sqrt(2 * E)
    assert np.all(d[1:, 3] >= 1)
    assert np.all(d[1:, 4] <= 1e-13)


def test_diagnostics_and_energy_identity():
    mesh, sp, x, c = case(1, (16, 16), 2, noise=0.0, nq=10)
    h = gpu_space(mesh, 2)
    h.set_upwind(1)
    E, dv, D = h.diagnostics(dev(x))
    assert abs(E - O.energy(sp, x)) <= 1e-13 * E
    assert abs(float(h.energy(dev(x))) - O.energy(sp, x)) <= 1e-13 * E
    assert dv <= 1e-12 * np.sqrt(2 * E)
    assert abs(dv - O.divergence_l2(sp, x)) <= 1e-13 * np.sqrt(2 * E)
    Dref = O.dissipation(sp, x, 1)
    assert abs(D - Dref) <= 1e-12 * Dref
    # divergence-free input: u.r(u) = D, up to the rounding of r and of the
    # inner product, whose terms sum to |u|.|r| = 2.3 here while D = 9.7e-6
    r = host(h.apply(dev(x)))
    assert abs(x @ r - D) <= 1e-13 * np.sum(np.abs(x * r))


@pytest.mark.parametrize("cfg,n,k,prec", [(1, (16, 16), 2, 1), (2, (4, 3, 3), 3, 1), (1, (16, 16), 2, 2),
                                         (2, (4, 3, 3), 3, 2), (2, (4, 3, 3), 3, 3), (3, (3, 3, 4), 5, 1),
                                         (3, (3, 3, 4), 5, 3)])
def test_substeps_mixed_precision(cfg, n, k, prec):
    """Mixed-precision substeps (FP32-MFMA or split-BF16 residual
    contractions, FP32 preconditioner contractions, FP64 state, mass operator
    and PCG): the PCG still meets the FP64 tolerance at every substep, and
    the chain stays within the contraction error of the oracle's FP64 chain.
    FP32-MFMA and hi/mid/lo: 1e-6.  hi/lo: its residual bound (3e-3, the
    apply tests) times the chain's relative increment sum_i |u_i+1 - u_i|/|u_i|
    (the state error is dt times the residual errors, summed), doubled."""
    mesh, sp, x, c = case(cfg, n, k)
    l = k - 1
    h = gpu_space(mesh, k)
    h.set_upwind(l)
    h.set_solver(rtol=1e-13, max_it=2000)
    u = dev(x)
    steps, dt = 5, 1e-3
    diag = host(h.substeps(u, dt, steps, prec=prec, diag=True))
    xs = O.substeps(sp, x, dt, steps, l, keep=True)
    incr = sum(rel_primal(sp, xs[i + 1], xs[i]) for i in range(steps))
    bound = 2 * 3e-3 * incr if prec == 2 else 1e-6
    print(f"mixed substeps prec={prec} cfg={cfg} k={k} its={diag[1:, 3]}")
    check_primal(sp, host(u), xs[-1], bound, f"mixed substeps prec={prec} cfg={cfg} k={k}", 4.0 * bound)
    assert np.all(diag[1:, 3] >= 1)
    assert np.all(diag[1:, 4] <= 1e-13)


def test_profile_counts_and_stride():
    """The library's launch timing counts one mass apply per PCG iteration
    that ran (launches left queued after convergence are not counted), and
    a stride times a subset of them."""
    mesh, sp, x, c = case(2, (4, 3, 3), 3)
    h = gpu_space(mesh, 3)
    h.set_upwind(2)
    h.set_solver(rtol=1e-13, max_it=2000, check_every=4)
    steps, dt = 3, 1e-3
    diag = host(h.substeps(dev(x), dt, steps, diag=True))
    its = int(diag[1:, 3].sum())
    h.profile(1)
    h.substeps(dev(x), dt, steps)
    n1, ms1 = h.profile_read("mass")
    h.profile(4)
    h.substeps(dev(x), dt, steps)
    n4, ms4 = h.profile_read("mass")
    h.profile(0)
    print(f"PCG iterations {its}: timed mass launches {n1} (stride 1), {n4} (stride 4)")
    assert n1 == its
    assert 1 <= n4 <= its // 4 + steps
    assert 0.5 < (ms4 / n4) / (ms1 / n1) < 2.0


@pytest.mark.parametrize("cfg,n,k", [(2, (4, 3, 3), 3), (3, (3, 4, 3), 4)])
def test_pcg_direction_ring_wraps(monkeypatch, cfg, n, k):
    """The PCG keeps its search directions in a ring and adds them to the
    solution at each host check; with a ring of 2 or 3 the chunks stop at
    the ring's capacity and the solve is bitwise the one with the full ring
    (the same updates in the same order); k = 4 runs the streamed-table
    mass kernels."""
    mesh, sp, x, c = case(cfg, n, k)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(sp.n_dof)
    ref = None
    for ring in (None, 3, 2):
        if ring is None:
            monkeypatch.delenv("HOPU_TEST_RING", raising=False)
        else:
            monkeypatch.setenv("HOPU_TEST_RING", str(ring))
        h = gpu_space(mesh, k)
        h.set_solver(rtol=1e-13, max_it=2000, check_every=5)
        w, its = h.mass_solve(dev(b), rtol=1e-13)
        w = host(w)
        h.close()
        if ref is None:
            ref, its_ref = w, its
            assert its > 6
        else:
            assert its == its_ref
            assert np.array_equal(w, ref), ring
    monkeypatch.delenv("HOPU_TEST_RING", raising=False)
    # and against the oracle's mass matrix
    assert rel_dual(sp, O.mass_apply(sp, ref), b) <= 1e-12


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 2), (3, 3)])
def test_divergence_closed_form(dim, k):
    """The GPU's ||div u||_L2 (hopu_diagnostics and the substeps' diagnostic
    row) for the parabola (0, y(1-y)[, 0]) on a graded, jittered, walled
    box equals the closed form sqrt(area / 3) to 1e-12."""
    from test_oracle_pins import walled_parabola_case
    sp, x, want, mesh = walled_parabola_case(dim, k)
    h = gpu_space(mesh, k)
    E, dv, D = h.diagnostics(dev(x))
    print(f"div closed form dim={dim} k={k}: {dv:.15e} vs {want:.15e}")
    assert abs(dv - want) <= 1e-12 * want
    d = host(h.substeps(dev(x), 1e-3, 0, diag=True))
    assert abs(d[0, 1] - want) <= 1e-12 * want


def test_warm_start_carry_across_calls():
    """hopu_set_warm_start(1): a trajectory advanced in two calls equals the
    one-call chain bit for bit (the extrapolation history continues), and
    the second call's first solve starts from the extrapolated guess
    (fewer iterations than from zero).  carry = 0: each call starts cold,
    and the states agree to the solve tolerance."""
    mesh, sp, x, c = case(2, (4, 3, 3), 3, noise=1e-3)
    h = gpu_space(mesh, 3)
    h.set_upwind(2)
    h.set_solver(rtol=1e-13, max_it=2000)
    dt = 5e-4
    one = dev(x)
    d1 = host(h.substeps(one, dt, 5, diag=True))
    two = dev(x)
    h.substeps(two, dt, 2)           # history starts here (this call cold)
    h.set_warm_start(True)
    d2 = host(h.substeps(two, dt, 3, diag=True))
    assert torch.equal(one, two)
    its_one, its_two = d1[1:, 3], d2[1:, 3]
    print("PCG iterations, one call", its_one, "second call", its_two)
    assert np.array_equal(its_one[2:], its_two)
    h.set_warm_start(False)
    cold = dev(x)
    h.substeps(cold, dt, 2)
    d3 = host(h.substeps(cold, dt, 3, diag=True))
    assert d3[1, 3] > d2[1, 3]
    check_primal(sp, host(cold), host(one), 1e-12, "cold restart vs one call")
    from paper_2408_06698_amd import _lib as L
    assert L.lib().hopu_set_warm_start(h.h, 2) == L.HOPU_EINVAL


def test_count_nonfinite():
    mesh, sp, x, c = case(2, (4, 3, 3), 3, noise=1e-3)
    h = gpu_space(mesh, 3)
    assert h.count_nonfinite(dev(x)) == 0
    v = x.copy()
    rng = np.random.default_rng(5)
    idx = rng.choice(sp.n_dof, 37, replace=False)
    v[idx[:20]] = np.nan
    v[idx[20:30]] = np.inf
    v[idx[30:]] = -np.inf
    assert h.count_nonfinite(dev(v)) == 37
    assert h.count_nonfinite(dev(x)) == 0     # the counter is cleared per call
