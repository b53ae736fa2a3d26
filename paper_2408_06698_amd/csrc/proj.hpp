// Launchers of the projection-step kernels (proj_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "kernels.hpp"

namespace hopu {

// Device data of the projection step: the multiplier-block index of every
// element facet (interior facets: their V_h facet id; walls: F + wall id),
// the mass tables in their row order, the Bm / Bm^t fragments and A^-1.
struct ProjDev {
  const int32_t* mfid;  // [E][d+1]
  int64_t FW;           // multiplier blocks (interior + wall facets)
  const double* mass_in;
  const double* prec_in;
  const double* prec_out;
  const double* b;      // [NBT][NMQ][64]
  const double* bt;     // [NMT][NQK][64]
  const double* ainv;   // [E][nQ][nQ]
};

// mode 0: facet-side contributions ([2][FW][nf]) of S_p ph, per-block
// partials of ph . S_p ph into part; mode 1: facet-side contributions of the
// right-hand side g from us; mode 2: out = us - u~ (V_h layout) from ph, us.
// Returns the number of blocks (partials) launched.  flag (nullable): the
// launch does nothing once *flag is set.
template <int D, int KK>
int launch_proj(hipStream_t s, int mode, const double* ph, const double* us, double* out, const DevMesh& mesh,
                const ProjDev& pj, double* part, const int* flag = nullptr);
template <int D, int KK>
void launch_proj_ainv(hipStream_t s, const DevMesh& mesh, const double* kab, double* ainv);

}  // namespace hopu
