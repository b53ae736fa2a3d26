// Implicit Stokes step of the operator splitting (paper section 2.2: the
// stress space Sigma_h, the skew space W_h, the facet space V^_h and the
// forms a_h, b_2h; section 2.3: eq. (MCS_step1), the static condensation of
// sigma and gamma, and the element-wise BDDC preconditioner).
//
// Element unknowns: the local velocity DoFs (facets, then interior), then
// the facet-tangential u^ unknowns (facet f, tangent c, mode j).  The
// stress is taken in the full trace-free P^{k+1} space with the nt-trace
// condition on interior facets imposed by Lagrange multipliers, which are
// condensed with sigma and gamma (same S_T as the constrained space).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

namespace hopu {

struct StokesDims {
  int dim = 0, k = 0;
  int nE = 0;     // trace-free matrix basis, d*d - 1
  int nG = 0;     // skew matrix basis, d(d-1)/2
  int nP1 = 0;    // dim P^{k+1}(T)
  int nPk = 0;    // dim P^k(T)
  int nsf = 0;    // full stress space nE * nP1
  int nft = 0;    // dim P^{k+1}(F)
  int ntop = 0;   // facet modes of degree exactly k + 1
  int ncons = 0;  // (d+1)(d-1) ntop constraint rows
  int n1 = 0;     // nG nPk + ncons (condensed multiplier-type rows)
  int n = 0;      // velocity DoFs per element
  int nf = 0;     // velocity DoFs per facet
  int nint = 0;   // interior velocity DoFs per element
  int nh = 0;     // local u^ unknowns (d+1)(d-1) nf
  int nx = 0;     // n + nh: unknowns of S_T
  int ng = 0;     // n1 + nx: rows of the element matrix G
  int nsd = 0;    // facet-side values: nf normal + (d-1) nf tangential
};
StokesDims stokes_dims(int dim, int k);

// Reference-element tables (FP64), laid out for the setup kernel.
//   Ea  [nE][d][d]   orthonormal trace-free basis (Frobenius)
//   Gc  [nG][d][d]   orthonormal skew basis
//   MpG [nPk][nP1]   int_T^ p_beta p_alpha (P^k modes against P^{k+1} modes)
//   TV  [nP1][n][d][d]  int_T^ d_r p_alpha phi^_{i,s}
//   Phi [d+1][nP1][nft] int_S^ p_alpha(x_f(s)) psi_m(s) ds (reference facet f)
//   Mref [n][n][d][d]   int_T^ phi^_{i,r} phi^_{j,s}
struct StokesTables {
  StokesDims sd;
  std::vector<double> Ea, Gc, MpG, TV, Phi, Mref;
};
bool make_stokes_tables(int dim, int k, StokesTables& t, std::string& err);

// Per-element record [E][STG]: J (row-major d x d, stride 3), J^-1 (stride 3),
// det J, then for each local facet f at 20 + 11 f: outward unit normal (3),
// unit tangents t_1, t_2 (3 each; t_1 from the facet's first two sorted
// vertices, t_2 = n_F x t_1 with n_F the sorted-vertex normal), |N_F| and
// 1.0 for an interior facet, 0.0 for a wall.
enum { STG = 64 };
void make_stokes_geometry(int dim, int64_t E, const std::vector<double>& xyz, const std::vector<double>& geo,
                          const std::vector<int32_t>& fid, std::vector<double>& out);

struct StokesDev {
  const double *Ea, *Gc, *MpG, *TV, *Phi, *Mref;
  const double* sgeo;       // [E][STG]
  const int32_t* fid;       // [E][d+1]
  const int32_t* facet_elem;  // [F][2]
  const int8_t* facet_local;  // [F][2]
  int64_t E, F, n_dof;
};

// Per-element storage of S_T and S_T^-1: the upper triangle packed by rows
// (row i holds entries j >= i at offset i nx - i (i - 1)/2), padded to a
// multiple of 8 doubles.
__host__ __device__ inline int64_t stokes_packed_stride(int nx) {
  return ((int64_t)nx * (nx + 1) / 2 + 7) / 8 * 8;
}
// S_T and S_T^-1 ([E][stokes_packed_stride(nx)] each); scratch holds
// nblocks * (ng * nsf + ng * ng) doubles.
int stokes_setup_blocks(const StokesDims& sd);
size_t stokes_setup_scratch(const StokesDims& sd);
// STinv32 non-null: S_T^-1 is stored in FP32 there instead of STinv.
void launch_stokes_setup(hipStream_t s, const StokesDims& sd, const StokesDev& dv, double nu, double dt,
                         double* ST, double* STinv, float* STinv32, double* scratch, int* bad);
// y = A x with A = S (inv = 0) or C_BDDC^-1 (inv = 1): element products
// (interior velocity rows into y, facet-side values into slot [E][d+1][nsd]),
// then the facet rows assembled from both sides.  The element matrices are
// read from A32 (FP32, FP64 arithmetic) when it is non-null, else from A.
void launch_stokes_gemv(hipStream_t s, const StokesDims& sd, const StokesDev& dv, const double* A, const float* A32,
                        int inv, const double* x, double* y, double* slot);
// per-block partials of a . b over n entries (npart of them)
int launch_stokes_dot(hipStream_t s, const double* a, const double* b, int64_t n, double* part);
// y += a x
void launch_stokes_axpy(hipStream_t s, double* y, const double* x, double a, int64_t n);
// p = z + b p
void launch_stokes_xpby(hipStream_t s, double* p, const double* z, double b, int64_t n);
// rhs: y[0, n_dof) = Mu/dt - r (r may be null), y[n_dof, n) = 0
void launch_stokes_rhs(hipStream_t s, double* y, const double* Mu, const double* r, double dt, int64_t n_dof,
                       int64_t n);

}  // namespace hopu
