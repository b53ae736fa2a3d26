#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "kernels.hpp"

namespace hopu {
enum { AUX_NPART = 1024 };
template <int D, int KK>
void launch_energy(hipStream_t s, const double* m, const DevMesh& mesh, double* part);
template <int D, int KK>
int64_t launch_div(hipStream_t s, const double* m, const DevMesh& mesh, const double* fdV, const double* wv,
                   double* part);
void launch_interp_points(hipStream_t s, int D, int nqs, const double* sp, int nqv, const double* xr,
                          const double* xyz, const DevMesh& mesh, double* pf, double* pv);
void launch_interpolate(hipStream_t s, int D, int nqs, int nf, const double* vf, const double* ws,
                        const double* psi, int nqv, int nint, const double* vv, const double* wv,
                        const double* qm, const DevMesh& mesh, double* x);
void launch_eval(hipStream_t s, int D, int n, int nf, int nint, int np, const double* x, const double* phi,
                 const DevMesh& mesh, double* out);
void launch_adapt(hipStream_t s, const double* eta_nd, int64_t F, const double* thr, int k, int8_t* lfac,
                  double* eta_out);
// count[0] = number of NaN / infinite entries of v[0, n)
void launch_count_nonfinite(hipStream_t s, const double* v, int64_t n, unsigned long long* count);
// measurement: register-only FP64 MFMA chains, blocks x 256 threads, out
// [blocks * 256]
void launch_mfma_f64_rate(hipStream_t s, double* out, int blocks, int iters);
}  // namespace hopu
