// Host-callable launchers of the device kernels (instantiated per order).
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.hpp"

namespace hopu {
template <typename T, int D, int KK>
void launch_modal(hipStream_t s, const double* x, T* m, const DevMesh& mesh, const T* frag);
template <typename T, int D, int KK>
void launch_elem(hipStream_t s, const T* m, double* r, double* slot, const DevMesh& mesh,
                 const DevTables<T>& tb, int terms, double* diss_part, double* eta_nd);
template <int D, int KK>
void launch_mass(hipStream_t s, int mode, const double* x, double* out, double* slot, const DevMesh& mesh,
                 const double* fin, const double* fout, const int* flag);
template <int D, int KK>
void launch_assemble(hipStream_t s, double* r, const double* slot, const DevMesh& mesh, const int* flag);
template <typename T, int D, int KK>
void launch_vjp(hipStream_t s, const T* mu_u, const T* mu_mu, double* out, double* slot, const DevMesh& mesh,
                const DevTables<T>& tb);
template <int D, int KK>
void launch_asm_dot(hipStream_t s, double* v, const double* slot, const double* w, const DevMesh& mesh, int64_t n,
                    const int* flag, double* part, int nblocks);
}  // namespace hopu
