// Host-side precompute for the HOPU convection library: quadrature, the
// reference dual basis of the normal-continuous velocity space, tabulated
// basis values, MFMA fragment tables, mesh topology and affine geometry.
// Plain C++17; no HIP types.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"

namespace hopu {

typedef long double ld;

// ------------------------------------------------------------ sizes
struct Sizes {
  int dim = 0, k = 0;
  int nP = 0;    // dim P^k(T)
  int nPs = 0;   // nP rounded up to a multiple of 4 (component stride)
  int nm = 0;    // modal rows per element = dim * nPs
  int n = 0;     // local dual DoFs = dim * nP
  int nf = 0;    // DoFs per facet = dim P^k(facet)
  int nfl = 0;   // facet DoFs per element = (dim+1) nf
  int nint = 0;  // interior DoFs per element
  int pv = 0, nqv = 0;  // volume rule points per direction / total
  int pf = 0, nqf = 0;  // facet rule points per direction / total
};
Sizes make_sizes(int dim, int k);
int dim_P(int dim, int k);

// ------------------------------------------------------------ quadrature
// Gauss-Jacobi nodes/weights for weight (1-x)^a (1+x)^b on [-1,1] by Newton
// iteration with polynomial deflation (long double).
void gauss_jacobi(int n, ld a, ld b, std::vector<ld>& x, std::vector<ld>& w);
// Collapsed rule on the reference dim-simplex (dim = 1,2,3); pts [nq][dim].
void simplex_rule(int dim, int npd, std::vector<ld>& pts, std::vector<ld>& w);

// ------------------------------------------------------------ bases
// Orthonormal (Dubiner) basis of P^k on the reference simplex at one point:
// val[nP], grad[nP][dim].
void dubiner(int dim, int k, const ld* x, ld* val, ld* grad);
// Facet polynomials psi_j at s (dim-1 coords): out[nf]; degree of each mode.
void facet_psi(int dim, int k, const ld* s, ld* out);
std::vector<int> facet_psi_degree(int dim, int k);
// Interior test fields q_m(x): out[nint][dim].
void interior_tests(int dim, int k, const ld* x, ld* out);
// Reference facet i: origin o[dim], edge matrix E[dim][dim-1] (column j =
// v_{j+1} - v_0 over the facet's vertices), unnormalised normal N[dim].
void ref_facet(int dim, int i, ld* o, ld* E, ld* N);

// Dual-basis matrices: D[j][(a,alpha)] = N_j(e_a p_alpha) (row-major n x n)
// and its inverse.
struct DualBasis {
  Sizes sz;
  std::vector<ld> D, Dinv;
};
bool make_dual_basis(int dim, int k, DualBasis& out, std::string& err);

// ------------------------------------------------------------ tables
// Reference tables at the operator quadrature points, FP64.
struct RefTables {
  Sizes sz;
  std::vector<double> wv;        // [nqv]
  std::vector<double> wf;        // [nqf]
  std::vector<double> V;         // [nqv][nP]
  std::vector<double> dV;        // [nqv][nP][dim]
  std::vector<double> Tr;        // [dim+1][nqf][nP]  p_alpha at facet points of local facet f
  std::vector<double> Psi;       // [nqf][nf]
  std::vector<int> psi_deg;      // [nf]
  std::vector<double> Kf;        // [dim+1][nf][nP]   sum_q wf psi_j p_alpha(x_f(q))
  std::vector<double> D, Dinv;   // [n][n] (dual x modal (a,alpha)) and inverse
  std::vector<double> xv;        // [nqv][dim] volume points
  std::vector<double> sf;        // [nqf][dim-1] facet points
  // projection step: Q_h = P^{k-1}, Bm[beta][rho(a, alpha)] = int_T^ d_a p_alpha q_beta
  int nQ = 0;
  std::vector<double> Bm;        // [nQ][nm]
};
bool make_ref_tables(int dim, int k, RefTables& t, std::string& err);

// Modal row layout: rho(a, alpha) = (alpha/4)*4*dim + 4*a + alpha%4.
// Dual row held at step s by lane group g (g = 0..3) in the mass kernels, or
// -1: for s < nf, groups g <= dim take row s of facet g; every other slot,
// in (s, g) order, takes the next interior row.
inline int mass_row(const Sizes& sz, int s, int g) {
  const int nfg = sz.dim + 1;  // facet groups
  if (s < sz.nf && g < nfg) return g * sz.nf + s;
  const int before = s < sz.nf ? s * (4 - nfg) : sz.nf * (4 - nfg) + (s - sz.nf) * 4;
  const int t = before + (s < sz.nf ? g - nfg : g);
  return t < sz.nint ? sz.nfl + t : -1;
}

inline int modal_row(int dim, int a, int alpha) {
  return (alpha / 4) * 4 * dim + 4 * a + (alpha % 4);
}

// MFMA fragment tables (A operands, lane order).  `rowmap` selects how a
// 16x16 output tile's rows sit in (register i, lane group g): FP64 MFMA puts
// row 4i+g in register i of group g, FP32 MFMA puts row 4g+i there.
enum RowMap { ROWMAP_F64 = 0, ROWMAP_F32 = 1 };
struct FragTables {
  // element kernel
  std::vector<double> modal;   // [NMT][NK][64]        Dinv rows rho, k = dual j
  std::vector<double> vol_V;   // [NQVT][NPK][64]      V[q][alpha]
  std::vector<double> vol_dVT; // [NQVT][4][dim][NAT][64]
  std::vector<double> fac_Tr;  // [dim+1][NQFT][NPK][64]
  std::vector<double> fac_TrT; // [dim+1][NQFT][4][NAT][64]
  std::vector<double> fac_K;   // [dim+1][NFJT][NPK][64]
  std::vector<double> fac_Psi; // [NQFT][NFK][64]
  std::vector<double> fac_PsiT;// [NQFT][4][NFJT][64]  (facet weights folded in)
  std::vector<double> fac_KT;  // [dim+1][NAT][NFK][64]
  std::vector<double> psi_n;   // [NQFT][NFK][64] FP64 values for the f64 MFMA, K = j (4 jk + lane group),
                               // rows permuted so that register i of lane group g holds this row map's point
  std::vector<double> dual;    // [NJT][dim][NAT][4][64]  Dinv^T by (a, alpha tile, reg)
  // vjp extras
  std::vector<double> vol_dV;  // [NQVT][dim][NPK][64]  d_b p_alpha at (q, alpha)
  std::vector<double> vol_VT;  // [NQVT][4][NAT][64]
  // mass / preconditioner sandwiches (modal rows in rho layout).  Their dual
  // rows follow mass_row(): lane group g holds facet g's rows, so a lane
  // touches one facet only.
  std::vector<double> mass_in;   // [NMT][NK][64]  Dinv rows rho, k = mass_row
  std::vector<double> mass_out;  // [NJT][NMQ][64] Dinv^T with k = rho quads
  std::vector<double> prec_in;   // [NMT][NK][64]  D^T rows rho, k = j
  std::vector<double> prec_out;  // [NJT][NMQ][64] D with k = rho quads
  // projection step (f64 layouts only)
  std::vector<double> proj_b;    // [NBT][NMQ][64]  Bm: rows beta, k = rho quads
  std::vector<double> proj_bt;   // [NMT][NQK][64]  Bm^T: rows rho, k = beta
  std::vector<double> proj_kab;  // [dim][dim][nQ][nQ]  sum_alpha Bm[.][rho(a,alpha)] Bm[.][rho(b,alpha)]
};
// tiles of the projection tables
inline int proj_nbt(int nQ) { return (nQ + 15) / 16; }
inline int proj_nqk(int nQ) { return (nQ + 3) / 4; }
struct FragDims {
  int NMT, NK, NQVT, NPK, NAT, NQFT, NFJT, NFK, NJT, NMQ;
};
FragDims frag_dims(const Sizes& s);
void make_frag_tables(const RefTables& t, RowMap rm, FragTables& f);

// Split-BF16 copies of the element kernel's FP32-layout tables (all but the
// modal and dual transforms, which run in FP64).  A table is
// viewed as [outer][nsteps][inner][64 lanes]; steps 4s .. 4s+3 of a lane
// become one 16x16x16 BF16 fragment, stored as ns bfloat16 terms (raw bits;
// hi, [mid,] lo by truncation of the FP32 value) laid out
// [outer][ceil(nsteps/4)][inner][64][ns][4]; steps past nsteps are zero.
struct BfTables {
  std::vector<uint16_t> vol_V, vol_dVT, fac_Tr, fac_TrT, fac_K, fac_Psi, fac_PsiT, fac_KT;
  std::vector<uint16_t> vol_dV, vol_VT;  // the transpose-Jacobian kernel's volume tables
};
std::vector<uint16_t> split_bf16_table(const std::vector<double>& t, int outer, int nsteps, int inner, int ns);
void make_bf16_tables(const FragTables& f32, const Sizes& s, int ns, BfTables& b);

// ------------------------------------------------------------ mesh
struct MeshData {
  int dim = 0;
  int64_t E = 0, F = 0, W = 0;
  std::vector<int64_t> vid;       // [E][d+1] sorted
  std::vector<double> xyz;        // [E][d+1][d] in sorted order
  std::vector<double> geo;        // [E][32]: J (row-major d x d), detJ, |N_F| (d+1),
                                  //          outward unit normals (d+1)*d
  std::vector<int32_t> fid;       // [E][d+1] interior facet id or -1
  std::vector<int32_t> nbr;       // [E][d+1] neighbour element or -1
  std::vector<int8_t> nbr_face;   // [E][d+1] neighbour's local facet or -1
  std::vector<int32_t> facet_elem;  // [F][2] lower element id first
  std::vector<int8_t> facet_local;  // [F][2]
};
bool build_mesh(int dim, int64_t E, const int64_t* elem_vid, const double* elem_xyz,
                MeshData& m, std::string& err);

// Element batches of 16 sharing the neighbour-facet signature
// (sig = sum_f code_f << 4f, code = neighbour local facet or 0xF for walls).
struct Batches {
  int64_t nb = 0;
  std::vector<int32_t> elem;   // [nb][16], -1 padding
  std::vector<int32_t> sig;    // [nb]
};
void make_batches(const MeshData& m, Batches& b);

}  // namespace hopu
