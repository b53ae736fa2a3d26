/* hopu.h -- C ABI of the MI355X HOPU explicit-convection library.
 *
 * What the library computes (Lederer, Mooslechner, Schoeberl, "High-order
 * projection-based upwind method for simulation of transitional turbulent
 * flows"):
 *   - the velocity space V_h of normal-continuous piecewise vector
 *     polynomials of degree k on affine simplices (section 2.2, eq.
 *     (disc_velspace); read as BDM_k, the full P^k per element), with
 *     normal velocity zero on wall facets;
 *   - the convection residual r(u)_i = c_h^HOPU(u, u, phi_i) of section 3.2,
 *     eq. (hopudefinition), in conservative volume form:
 *       r_i = - sum_T int_T (u x u) : grad phi_i
 *             + sum_{E in F^I} int_E (u.n) <u>.[[phi_i]]
 *               + 1/2 |u.n| (I - Pi^l)[[u]] . (I - Pi^l)[[phi_i]]
 *     (Pi^l: facet-wise L2 projection onto degree <= l; l = -1 gives the
 *     standard upwind of eq. (upwind), l = k the central flux);
 *   - the velocity mass matrix M (M_uu = M/dt in the matrix form of the
 *     splitting, section 2.3) and its inverse by PCG with the element-wise
 *     BDDC preconditioner without primal constraints, R blockdiag(M_T)^-1 R^t,
 *     R the averaging operator (section 2.3);
 *   - explicit convection substeps u <- u - dt M^-1 r(u) (the explicit part
 *     of step 1, eq. (MCS_step1));
 *   - transpose Jacobians of r and of the substep chain;
 *   - the two steps of the operator splitting (section 2.3): the projection
 *     of eq. (MCS_step2) (hopu_project) and the implicit Stokes step of eq.
 *     (MCS_step1) with its static condensation and element-wise BDDC
 *     (hopu_stokes_*).
 *
 * Coefficient vectors ("global layout"): FP64, length n_dof =
 *   [interior-facet block: facets in lexicographic order of their sorted
 *    vertex-id tuple, n_facet_dof each] ++ [element block: elements in input
 *    order, n_interior_dof each].
 * Facet DoF j of facet F: int over the reference facet of (u . n_F) psi_j,
 * n_F the unit normal (x_b - x_a) x (x_c - x_a) (3D) or rot(x_b - x_a) (2D)
 * from the facet's vertices in ascending id order, psi_j orthonormal facet
 * polynomials; interior DoFs: moments of the contravariant Piola pull-back
 * against gradients of monomials and Koszul fields, scaled by
 * |det J|^{-(d-1)/d}.  Residual vectors are dual vectors in the same layout.
 *
 * Conventions for every call:
 *   - returns hopu_status; never aborts; HIP errors map to HOPU_EHIP with the
 *     HIP error string in hopu_last_error();
 *   - vectors marked "dev" are HIP device pointers (for example a torch
 *     tensor's data_ptr() on ROCm) owned by the caller; "host" pointers are
 *     host memory owned by the caller;
 *   - work is queued on the context's stream; calls marked "syncs" wait for
 *     it before returning; others are asynchronous;
 *   - a context is not thread-safe; calls on one context must not overlap.
 *
 * Test hooks (environment variables, for tests of failure and wrap-around
 * paths; unset in normal use): HOPU_TEST_FAIL_ALLOC=1 makes every device
 * allocation of the library fail with HOPU_ENOMEM; HOPU_TEST_RING=h sets
 * the PCG search-direction ring to h vectors (see hopu_create).
 */
#ifndef HOPU_H
#define HOPU_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hopu_ctx_s* hopu_ctx;

typedef enum {
  HOPU_OK = 0,
  HOPU_EINVAL = -1,       /* bad argument (null pointer, k out of range, ...) */
  HOPU_EMESH = -2,        /* malformed mesh: repeated vertex, det J = 0,
                             facet in > 2 elements, too few periodic cells */
  HOPU_ENOMEM = -3,       /* device allocation failed */
  HOPU_EHIP = -4,         /* HIP runtime error */
  HOPU_ENOCONV = -5,      /* PCG did not reach the tolerance in max_it */
  HOPU_EUNSUPPORTED = -6  /* valid request the library does not implement */
} hopu_status;

typedef enum {
  HOPU_FP64 = 0,       /* all contractions in FP64 (MFMA f64) */
  HOPU_FP32_MFMA = 1,  /* basis contractions on FP32 MFMA with FP32 accumulation
                          inside a tile and FP64 across tiles; state, mass
                          inverse and diagnostics stay FP64 */
  HOPU_BF16X2 = 2,     /* the same contractions on BF16 MFMA, each operand split
                          into hi + lo bfloat16 terms (hh + hl + lh kept, about
                          16 significant bits); FP32 accumulation inside a
                          tile, FP64 across tiles.  Apply, substeps and the
                          adjoint calls */
  HOPU_BF16X3 = 3      /* hi + mid + lo split (hh, hm, mh, hl, mm, lh kept: the
                          24 bits of the FP32 value); otherwise as HOPU_BF16X2 */
} hopu_precision;

enum { HOPU_TERM_VOLUME = 1, HOPU_TERM_CENTRAL = 2, HOPU_TERM_UPWIND = 4, HOPU_TERM_ALL = 7 };

/* Build the space: dim 2|3, order k 1..5 (k=6 returns HOPU_EUNSUPPORTED),
 * elem_vid host int64 [n_elems][dim+1] vertex ids with periodic images
 * identified; elem_xyz host double [n_elems][dim+1][dim] unwrapped vertex
 * coordinates of each element; hip_stream a hipStream_t (NULL = default).
 * Host work: topology, geometry, tables; then device allocation and copies.
 * Device memory: about 15 vectors of n_dof doubles, the element workspaces
 * and the PCG search-direction ring (min(64, 32 GB / (8 n_dof)) vectors, at
 * least 4; the environment variable HOPU_TEST_RING = h, 2 <= h <= 64, read
 * here, sets h vectors instead, for tests of the ring's wrap-around).
 * Syncs. */
hopu_status hopu_create(hopu_ctx* out, int dim, int k, int64_t n_elems,
                        const int64_t* elem_vid, const double* elem_xyz,
                        void* hip_stream);

/* Sizes of the space; any output pointer may be NULL. */
hopu_status hopu_sizes(hopu_ctx ctx, int64_t* n_dof, int64_t* n_facets,
                       int64_t* n_wall_facets, int* n_loc, int* n_facet_dof,
                       int* n_interior_dof);

/* HOPU projection degree (section 3.2): l_global in -1..k applies to every
 * facet; l_per_facet_dev (dev int8 [n_facets], nullable) overrides it per
 * facet.  The pointer is kept and read by later calls. */
hopu_status hopu_set_upwind(hopu_ctx ctx, int l_global, const int8_t* l_per_facet_dev);

/* Adaptive HOPU order (end of section 3.2).  The jump indicator of a facet
 * is eta_E = int_E |(I - Pi^l)[[u]]| ds / int_E |<u>| ds with the facet's
 * current order l; given thresholds eta_0 < ... < eta_k (eta_{k+1} = 1) the
 * order becomes l = i for eta_i < eta <= eta_{i+1}, -1 (standard upwind) for
 * eta <= eta_0 and k for eta > 1.  A facet with <u> = 0 gets eta = 0 if its
 * projected jump is zero, else +inf.
 * hopu_jump_indicator: eta per interior facet, eta_dev dev double [n_facets].
 * hopu_set_adaptive: every > 0 enables the adaptive order with host
 *   thresholds[k+1] and initial order l_initial for every facet (the context
 *   owns the per-facet order array); hopu_substeps then recomputes the orders
 *   from the current state before every `every`-th substep (steps 0, every,
 *   ...).  every <= 0 disables it; hopu_set_upwind also disables it.
 * hopu_adapt_upwind: recompute the orders from u now. */
hopu_status hopu_jump_indicator(hopu_ctx ctx, const double* u, double* eta_dev);
hopu_status hopu_set_adaptive(hopu_ctx ctx, int every, int n_thresholds, const double* thresholds, int l_initial);
hopu_status hopu_adapt_upwind(hopu_ctx ctx, const double* u);
/* Copy the context's current per-facet orders (adaptive mode) to l_dev
 * (dev int8 [n_facets]).  Asynchronous. */
hopu_status hopu_get_facet_orders(hopu_ctx ctx, int8_t* l_dev);

/* PCG controls for mass solves inside substeps and their adjoints:
 * stop when sqrt(r.z) <= rtol sqrt(b.Pb) (preconditioned residual norm);
 * check_every: iterations between host reads of the convergence flag. */
hopu_status hopu_set_solver(hopu_ctx ctx, double rtol, int max_it, int check_every);

/* r = C(u) u: the convection residual (dual vector).  u, r dev [n_dof].
 * terms: bitmask of HOPU_TERM_*.  Asynchronous: only kernel launches on the
 * context's stream (no allocation, copy, memset or synchronisation while
 * per-kernel timing is off), so the call may be captured into a HIP graph
 * on that stream. */
hopu_status hopu_convection_apply(hopu_ctx ctx, const double* u, double* r,
                                  int terms, hopu_precision prec);

/* y = M u (dev [n_dof] each).  Asynchronous. */
hopu_status hopu_mass_apply(hopu_ctx ctx, const double* u, double* y);

/* w = M^-1 r by PCG (FP64).  w dev [n_dof] holds the initial guess on entry.
 * rtol <= 0 selects the context default; *iters (host, nullable) receives the
 * iteration count.  Syncs.  HOPU_ENOCONV if max_it is reached. */
hopu_status hopu_mass_solve(hopu_ctx ctx, const double* r, double* w,
                            double rtol, int max_it, int* iters);

/* Projection step of the operator splitting (paper section 2.3, eq.
 * (MCS_step2), update eq. (UpdateStep) read as u_new = u* - u~): the
 * hybrid-mixed problem for (u~, p, p^) in the broken velocity space x
 * P^{k-1} per element x P^k per facet (walls included) is condensed onto the
 * facet multipliers p^ and solved by CG (FP64) to
 * ||r|| <= rtol (||g||^2 + ||u*_F||^2)^1/2 (g the condensed right-hand side,
 * u*_F the facet block of u*, in the same units), then
 * u~ is recovered element by element.  u_new is divergence-free and lies in
 * V_h.  ustar, unew: dev [n_dof], distinct (else HOPU_EINVAL).  rtol > 0,
 * max_it >= 1; *iters (host, nullable) receives the CG iteration count.
 * The first call allocates the step's workspace (E dim P^{k-1}^2 + (4 + H)
 * (F + W) n_f doubles; H, the CG's search-direction ring, is
 * min(17, 8 GB / (8 (F + W) n_f)) and at least 4) and computes the element
 * matrices A^-1; later calls allocate nothing.  Syncs.  HOPU_ENOCONV if
 * max_it is reached (unew is still written from the last iterate). */
hopu_status hopu_project(hopu_ctx ctx, const double* ustar, double* unew,
                         double rtol, int max_it, int* iters);

/* Measurement helper (no context): the FP64 MFMA rate the current device
 * sustains with independent 16x16x4 accumulation chains held in registers
 * (no memory traffic), blocks_per_cu (1..8) blocks of four waves per compute
 * unit, i.e. that many waves per SIMD.  The practical ceiling against which
 * the FP64 kernels' MFMA rates can be read.  *tflops (host) receives the
 * rate.  Allocates a small buffer; syncs the default stream. */
hopu_status hopu_mfma_f64_rate(int blocks_per_cu, double* tflops);

/* n_steps explicit substeps u <- u - dt M^-1 r(u), in place on u (dev).
 * diag_dev (dev double [n_steps+1][5], nullable): per state energy
 * 1/2 u.Mu, ||div u||_L2, upwind dissipation, PCG iterations of the solve
 * that produced it, final preconditioned relative residual.  Syncs. */
hopu_status hopu_substeps(hopu_ctx ctx, double* u, double dt, int n_steps,
                          hopu_precision prec, double* diag_dev);

/* carry = 1: hopu_substeps starts the PCG initial-guess extrapolation from
 * the solutions of the previous hopu_substeps call on this context (for a
 * caller that advances one trajectory with one dt in several calls);
 * carry = 0 (default): every call starts from a zero guess.  Either way the
 * solves meet the tolerance; only the iteration counts differ. */
hopu_status hopu_set_warm_start(hopu_ctx ctx, int carry);

/* out = J_r(u)^T mu (dev [n_dof] each), the derivative of the residual of
 * eq. (hopudefinition) with respect to the state, transposed.  |u.n| is not
 * differentiable at 0: its derivative is taken as sgn(u.n) with sgn(0) = 0,
 * u.n within 1e-8 |<u>| of zero (rounding noise of a field tangential to
 * the facet) counting as zero.  The reduced forms evaluate u.n for that
 * decision in FP64 from the state's facet DoFs.  Asynchronous. */
hopu_status hopu_convection_vjp(hopu_ctx ctx, const double* u, const double* mu,
                                double* out, hopu_precision prec);

/* Reverse pass of n_steps substeps from u0: lam_0 = (d u_N / d u_0)^T lam_N.
 * Checkpoints every ckpt_every states and recomputes each segment.
 * ws dev workspace of ws_bytes >= hopu_substeps_vjp_workspace() bytes.
 * Syncs. */
int64_t hopu_substeps_vjp_workspace(hopu_ctx ctx, int n_steps, int ckpt_every);
hopu_status hopu_substeps_vjp(hopu_ctx ctx, const double* u0, double dt, int n_steps,
                              int ckpt_every, const double* lam_N, double* lam_0,
                              hopu_precision prec, void* ws, int64_t ws_bytes);

/* Number of NaN or infinite entries of v (dev [n_dof]) into *count (host):
 * the check for a state or residual that has blown up (every other call
 * propagates non-finite values without a status).  Syncs. */
hopu_status hopu_count_nonfinite(hopu_ctx ctx, const double* v, int64_t* count);

/* Kinetic energy 1/2 u.Mu of u (dev [n_dof]) into energy_dev (dev, one
 * double), FP64.  Asynchronous (the loss of the adjoint workload). */
hopu_status hopu_energy(hopu_ctx ctx, const double* u, double* energy_dev);

/* Energy 1/2 u.Mu, ||div u_h||_L2 and the upwind dissipation
 * sum_E int 1/2 |u.n| |(I-Pi^l)[[u]]|^2 (host scalars, nullable).  Syncs. */
hopu_status hopu_diagnostics(hopu_ctx ctx, const double* u, double* energy,
                             double* div_l2, double* dissipation);

/* Interpolation of a field sampled by the caller.  hopu_interp_points writes
 * the physical sample points for a rule of n1d points per direction:
 * pts_facet dev [n_facets][n1d^(d-1)][d], pts_vol dev [n_elems][n1d^d][d].
 * hopu_interpolate turns field values at those points (same shapes) into
 * coefficients u (dev [n_dof]) with the DoF functionals. */
hopu_status hopu_interp_points(hopu_ctx ctx, int n1d, double* pts_facet, double* pts_vol);
hopu_status hopu_interpolate(hopu_ctx ctx, int n1d, const double* vals_facet,
                             const double* vals_vol, double* u);

/* Evaluate u at reference points: ref_pts host [n_pts][d],
 * vals dev [n_elems][n_pts][d].  Asynchronous. */
hopu_status hopu_eval(hopu_ctx ctx, const double* u, int n_pts,
                      const double* ref_pts, double* vals);

/* hopu_eval without allocating: for callers that cannot allocate device or
 * host memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments and result as
 * hopu_eval; the basis table at the points goes to a scratch array the
 * library keeps in each GPU's memory for the life of the process (1 MiB,
 * i.e. n_pts * n_loc * dim <= 131072 doubles: at most 260 points at 3D
 * k = 5); larger n_pts return HOPU_EINVAL with the limit in the message.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on
 * one GPU (from several threads or streams) race.  Syncs. */
hopu_status hopu_eval_noalloc(hopu_ctx ctx, const double* u, int n_pts,
                              const double* ref_pts, double* vals);

/* Per-kernel timing with HIP events attached to launches of the main kernels
 * (for benchmarks and roofline reports).  hopu_profile_enable(ctx, s, n),
 * s >= 1, starts recording every s-th launch of each kernel kind (s = 1:
 * every launch), up to n recorded launches, and resets earlier records;
 * (ctx, 0, 0) stops.  Events on a dispatch delay it by a few microseconds,
 * so a stride keeps a timed run close to an uninstrumented one.  Launches
 * that a converged PCG left queued are not counted.  hopu_profile_read
 * returns, for one kernel kind (0 element/convection kernel, 1 mass apply
 * inside PCG, 2 preconditioner inside PCG, 3 dual->modal transform,
 * 4 transpose-Jacobian kernel, 5 mass/preconditioner applies outside the
 * PCG loop, 6 the Stokes step's element product with S_T, 7 the same with
 * S_T^-1), the number of recorded launches and their summed duration in
 * ms.  Both sync. */
hopu_status hopu_profile_enable(hopu_ctx ctx, int enable, int max_launches);
hopu_status hopu_profile_read(hopu_ctx ctx, int kind, int64_t* launches, double* total_ms);

/* Message of the last failed call on ctx (or of the last failed
 * hopu_create when ctx is NULL); valid until the next call. */
const char* hopu_last_error(hopu_ctx ctx);

/* Frees everything the context owns.  NULL-safe. */
void hopu_destroy(hopu_ctx ctx);

/* ---- implicit Stokes step (paper section 2.2: the stress space Sigma_h of
 * trace-free P^{k+1} matrices with nt-traces of degree k on interior facets,
 * the skew space W_h = P^k, the tangential facet space V^_h = P^k with u^ = 0
 * on walls, the forms a_h and b_2h; section 2.3: eq. (MCS_step1), its matrix
 * form, the static condensation S = A - B M^-1 B^t of sigma and gamma, and
 * PCG with the element-wise BDDC preconditioner C^-1 = R S_BDDC^-1 R^t,
 * without primal constraints).  Built for k <= 4 in 2D and 3D
 * (HOPU_EUNSUPPORTED otherwise).
 *
 * Unknown vector X (device, FP64, n_total = n_dof + n_uhat entries): the
 * velocity DoFs in the layout of the other calls, then u^ per interior facet
 * (facet ascending, tangent c = 0..d-2, mode j = 0..n_f-1 fastest) with
 * u^|_F(x(s)) = sum_c sum_j u^_{F,c,j} psi_j(s) t_{F,c}: psi_j the facet
 * polynomials of the velocity DoFs on the facet's sorted-vertex
 * parametrisation, t_{F,1} = (x_b - x_a)/|x_b - x_a| from its first two
 * sorted vertices, t_{F,2} = n_F x t_{F,1} (3D).  div of a matrix field is
 * row-wise; sigma_nt = sigma n - (n . sigma n) n.
 *
 * hopu_stokes_sizes: n_total, n_uhat and the unknowns per element of S_T
 *   (any pointer may be NULL).
 * hopu_stokes_setup: nu > 0, dt > 0; flags 0 or HOPU_STOKES_FP32_PRECOND (keep
 *   S_T^-1 in FP32: the preconditioner's element products read half the
 *   bytes and compute in FP64; S, the vectors and the inner products stay
 *   FP64, so the step meets the same tolerance).  Builds on the GPU, per element, S_T on
 *   its velocity and u^ unknowns and S_T^-1, and keeps both in device memory
 *   (their upper triangles: about E nx^2 doubles, nx from hopu_stokes_sizes).  Allocates on its first
 *   call (HOPU_ENOMEM if that fails) and a set-up scratch for each call;
 *   HOPU_EINVAL if an element matrix is not positive definite.  Re-call it
 *   when nu or dt changes.
 * hopu_stokes_apply: y = S x (assembled; x and y distinct, n_total each).
 * hopu_stokes_precond: y = C^-1 x = R S_BDDC^-1 R^t x (R averages the two
 *   copies of every facet unknown).
 * hopu_stokes_step: one step of eq. (MCS_step1) from u^n (n_dof entries):
 *   PCG on S X = [M u^n/dt - r(u^n); 0] with C^-1, where r is the FP64
 *   convection residual of hopu_convection_apply with the context's upwind
 *   setting when flags has HOPU_STOKES_CONVECTION and zero otherwise.  The
 *   PCG starts from X = 0, or from the contents of x when flags has
 *   HOPU_STOKES_GUESS (in a time loop [u^n; u^ of the previous step] is a
 *   good guess).  Writes X = [u*; u^] to x (n_total entries) and the
 *   iteration count to *iters (may be NULL).  Stops when the C^-1 norm of
 *   the residual falls below rtol times the C^-1 norm of the right-hand
 *   side; HOPU_ENOCONV after max_it iterations (x then holds the last
 *   iterate); HOPU_EINVAL for other flag bits.  Synchronises the context's
 *   stream.
 * Every Stokes call except hopu_stokes_sizes needs hopu_stokes_setup first
 * (HOPU_EINVAL otherwise). */
hopu_status hopu_stokes_sizes(hopu_ctx ctx, int64_t* n_total, int64_t* n_uhat, int* n_elem_unknowns);
enum { HOPU_STOKES_FP32_PRECOND = 1 };
hopu_status hopu_stokes_setup(hopu_ctx ctx, double nu, double dt, int flags);
hopu_status hopu_stokes_apply(hopu_ctx ctx, const double* x, double* y);
hopu_status hopu_stokes_precond(hopu_ctx ctx, const double* x, double* y);
enum { HOPU_STOKES_CONVECTION = 1, HOPU_STOKES_GUESS = 2 };
hopu_status hopu_stokes_step(hopu_ctx ctx, const double* un, int flags, double* x, double rtol,
                             int max_it, int* iters);

/* ---- host-only inspection (no HIP calls; used by CPU tests) ------------
 * hopu_host_tables: reference tables for (dim, k): which = 0 volume points
 * [nqv][d], 1 volume weights, 2 V [nqv][nP] (internal modal basis), 3 facet
 * points [nqf][d-1], 4 facet weights, 5 psi [nqf][nf], 6 D [n][n],
 * 7 Dinv [n][n]; the element kernel's fragment tables in the FP32 register
 * layout: 8 vol_dVT [NQVT][4][d][NAT][64], 11 fac_Tr [d+1][NQFT][NPK][64],
 * 13 vol_dV [NQVT][d][NPK][64], 14 vol_VT [NQVT][4][NAT][64] (the last two
 * are the transpose-Jacobian kernel's volume tables), and split-BF16 copies
 * as raw bfloat16 bit patterns (one per double): 9 vol_dVT hi/lo, 10 vol_dVT
 * hi/mid/lo, 12 fac_Tr hi/mid/lo, 15 vol_dV hi/mid/lo, 16 vol_VT
 * hi/mid/lo, laid out [outer][ceil(steps/4)][inner][64][terms][4]; the
 * Stokes step's reference tables: 20 Ea [d*d-1][d][d] (orthonormal
 * trace-free basis), 21 Gc [d(d-1)/2][d][d] (orthonormal skew basis), 22 MpG
 * [dim P^k][dim P^{k+1}], 23 TV [dim P^{k+1}][n][d][d], 24 Phi
 * [d+1][dim P^{k+1}][dim P^{k+1}(F)], 25 Mref [n][n][d][d] (the last four
 * with the P^{k+1} basis scaled to unit norm).  Writes at most cap
 * doubles; returns the count or < 0.
 * hopu_host_mesh: topology/geometry of a mesh: which = 0 fid int32
 * [E][d+1], 1 nbr int32, 2 nbr_face (as int32), 3 geometry double
 * [E][32], 4 facet_elem int32 [F][2] (free facets only; a wall side has
 * nbr -1), 5 batches int32 [nb][16], 6 the Stokes step's element frames
 * double [E][64] (J, J^-1 with row stride 3, det J at 18, then per local
 * facet f at 20 + 11 f: outward unit normal, tangents t_1, t_2, |N_F|,
 * 1 interior / 0 wall).  Writes at most cap entries; returns
 * the array's full length (which may exceed cap), -1 for bad arguments, -2
 * for a mesh the builder rejects.
 * hopu_host_sizes: sizes of the space for (dim, k): which = 0 n_loc, 1 n_f
 * (DoFs per facet), 2 n_int (interior DoFs per element), 3 dim P^k, 4 volume
 * points, 5 facet points; -1 for an unsupported (dim, k) or which. */
int64_t hopu_host_tables(int dim, int k, int which, double* out, int64_t cap);
int64_t hopu_host_mesh(int dim, int64_t n_elems, const int64_t* elem_vid,
                       const double* elem_xyz, int which, void* out, int64_t cap);
int64_t hopu_host_sizes(int dim, int k, int which);

#ifdef __cplusplus
}
#endif
#endif
