// Host-callable launchers of the device kernels (instantiated per order).
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.hpp"

namespace hopu {
// frag: the FP64 modal table (the transform is FP64 for every storage type)
template <typename T, int D, int KK>
void launch_modal(hipStream_t s, const double* x, T* m, const DevMesh& mesh, const double* frag);
template <typename T, int D, int KK>
void launch_elem(hipStream_t s, const T* m, double* r, double* slot, const DevMesh& mesh,
                 const DevTables<T>& tb, int terms, double* diss_part, double* eta_nd);
// m = Dinv S x (rho layout) by the persistent mass kernel's gather and first
// contraction, stored as double or float (f32); mass_in table; fs: the
// facet-side buffer (only its trash slots are written).  Returns false for
// orders whose table does not fit in LDS (then launch_modal does it).  x
// must be 16-byte aligned.
template <int D, int KK>
bool launch_modal_mass(hipStream_t s, const double* x, void* m, bool f32, double* fs, const DevMesh& mesh,
                       const double* fin);
// The element kernel with split-BF16 contractions (NS = 2: hi/lo, 3:
// hi/mid/lo), FP32 modal coefficients and the regrouped tables.
template <int NS, int D, int KK>
void launch_elem_bf(hipStream_t s, const float* m, double* r, double* slot, const DevMesh& mesh,
                    const DevTables<BfPack<NS>>& tb, int terms, double* diss_part);
// y = M x (mode 0) or the preconditioner applied to x (mode 1): interior rows
// into out, facet rows as one contribution per side into fs ([2][F][NF]);
// with part set, also the per-block partials of x . y.  With fin32/fout32
// set, mode 1 runs its contractions in FP32 MFMA (orders whose tables fit in
// LDS).  Returns the number of blocks launched (= partials written).
template <int D, int KK>
int launch_mass(hipStream_t s, int mode, const double* x, double* out, double* fs, const DevMesh& mesh,
                const double* fin, const double* fout, const int* flag, double* part, const float* fin32 = nullptr,
                const float* fout32 = nullptr);
// facet rows v[0, nfl) = fs[0][.] + fs[1][.]
void launch_fs_assemble(hipStream_t s, double* v, const double* fs, int64_t nfl, const int* flag);
template <int D, int KK>
void launch_assemble(hipStream_t s, double* r, const double* slot, const DevMesh& mesh, const int* flag);
// udual: the FP64 state (its facet DoFs give u.n); psi_n: the f64 MFMA
// table of the facet polynomials in the point order of T's row map
template <typename T, int D, int KK>
void launch_vjp(hipStream_t s, const T* mu_u, const T* mu_mu, double* out, double* slot, const DevMesh& mesh,
                const DevTables<T>& tb, const double* udual, const double* psi_n);
// the transpose-Jacobian kernel with split-BF16 contractions (as launch_elem_bf)
template <int NS, int D, int KK>
void launch_vjp_bf(hipStream_t s, const float* mu_u, const float* mu_mu, double* out, double* slot,
                   const DevMesh& mesh, const DevTables<BfPack<NS>>& tb, const double* udual, const double* psi_n);
}  // namespace hopu
