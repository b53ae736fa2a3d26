"""FP64 CPU oracle for the HOPU explicit-convection hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
bench's CPU-baseline leg may import this package.  The library under
`paper_2408_06698_amd` never imports, links or calls it, and it imports
nothing from the library.

What it computes, from the paper's definitions (Lederer, Mooslechner,
Schoeberl, "High-order projection-based upwind method for simulation of
transitional turbulent flows"):

  * the normal-continuous H(div) velocity space V_h (section 2.2, eq.
    (disc_velspace)) on affine simplices, read as full P^k vector
    polynomials per element with continuous normal component (BDM_k);
  * the HOPU convection form (section 3.2, eq. (hopudefinition)) in its
    conservative volume form (u x u):grad v plus the facet flux
    (u.n)<u>.[[v]] + 1/2 |u.n| (I - Pi^l)[[u]] . (I - Pi^l)[[v]], and the
    paper's advective form for cross-checks; l = -1 gives the standard upwind
    of eq. (upwind), l = k the central flux;
  * the velocity mass matrix M (M_uu = M / dt in the matrix form of step 1,
    section 2.3) and its inverse by a direct or CG solve;
  * the explicit convection substep u <- u - dt M^{-1} r(u) (the explicit part
    of step 1, eq. (MCS_step1));
  * energy, divergence and upwind-dissipation diagnostics;
  * the transpose Jacobian of r and of the substep chain;
  * the projection step (section 2.3, eq. (MCS_step2));
  * the implicit Stokes step (section 2.2 spaces Sigma_h, W_h, V^_h and forms
    a_h, b_2h; section 2.3 eq. (MCS_step1), its static condensation and the
    element-wise BDDC preconditioner).

Everything is evaluated in physical coordinates with element and facet loops
(vectorised over batches).  Parity status of each function is stated in its
docstring, and so is each reading taken where the paper does not fix an
item (the quadrature rule, the basis, the adaptive thresholds' ties).
"""
from . import quadrature, basis, mesh, space, operator, projection, stokes  # noqa: F401
