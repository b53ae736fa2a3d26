// Diagnostics (energy, divergence), interpolation and evaluation kernels.
#include <algorithm>

#include "aux.hpp"
#include "kernels.hpp"

namespace hopu {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// 1/2 u.Mu = 1/2 sum_T m^T (G (x) I) m / |det J| (orthonormal modal basis)
template <int D, int KK>
__global__ __launch_bounds__(256) void k_energy(const double* __restrict__ m, DevMesh mesh, double* part) {
  using C = Cfg<D, KK>;
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mesh.E; e += (int64_t)gridDim.x * 256) {
    const double* g = mesh.geo + e * GEO_STRIDE;
    double Gm[D][D];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) {
        double t = 0;
        for (int r = 0; r < D; ++r) t += g[r * D + a] * g[r * D + b];
        Gm[a][b] = t;
      }
    double es = 0.0;
    for (int al = 0; al < C::NP; ++al) {
      double v[D];
      for (int a = 0; a < D; ++a) v[a] = m[e * C::NM + (al / 4) * 4 * D + 4 * a + (al % 4)];
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) es += v[a] * Gm[a][b] * v[b];
    }
    s += 0.5 * es / fabs(g[GEO_DET]);
  }
  const double t = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ||div u||^2 = sum_T int (div^ u^)^2 / |det J| dx^, div^ u^ by MFMA over alpha
template <int D, int KK>
__global__ __launch_bounds__(256) void k_div(const double* __restrict__ m, DevMesh mesh,
                                             const double* __restrict__ fdV, const double* __restrict__ wv,
                                             double* part) {
  using C = Cfg<D, KK>;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nw = (mesh.E + 15) / 16;
  double s = 0.0;
  if (wave < nw) {
    const int64_t e = wave * 16 + c;
    const bool valid = e < mesh.E;
    const int64_t ee = valid ? e : 0;
    double mB[D][C::NPK];
    for (int a = 0; a < D; ++a)
      for (int kk = 0; kk < C::NPK; ++kk) mB[a][kk] = m[ee * C::NM + kk * 4 * D + 4 * a + g];
    for (int qt = 0; qt < C::NQVT; ++qt) {
      d4 dv = {0, 0, 0, 0};
      for (int a = 0; a < D; ++a)
        for (int kk = 0; kk < C::NPK; ++kk)
          dv = __builtin_amdgcn_mfma_f64_16x16x4f64(fdV[((qt * D + a) * C::NPK + kk) * 64 + lane], mB[a][kk], dv,
                                                    0, 0, 0);
      for (int i = 0; i < 4; ++i) {
        const int q = 16 * qt + 4 * i + g;
        if (q < C::NQV) s += wv[q] * dv[i] * dv[i];
      }
    }
    s = valid ? s / fabs(mesh.geo[ee * GEO_STRIDE + GEO_DET]) : 0.0;
  }
  for (int w = 32; w >= 1; w >>= 1) s += __shfl_xor(s, w, 64);
  if (lane == 0 && wave < nw) part[wave] = s;
}

__global__ void k_interp_points_facet(int D, int nqs, const double* __restrict__ s, const double* __restrict__ xyz,
                                      DevMesh mesh, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mesh.F * nqs) return;
  const int64_t F = t / nqs;
  const int q = (int)(t - F * nqs);
  const int64_t T = mesh.facet_elem[2 * F];
  const int i = mesh.facet_local[2 * F];
  int lv[3], c = 0;
  for (int v = 0; v <= D; ++v) if (v != i) lv[c++] = v;
  const double* X = xyz + T * (D + 1) * D;
  for (int a = 0; a < D; ++a) {
    double x = X[lv[0] * D + a];
    for (int j = 0; j < D - 1; ++j) x += s[q * (D - 1) + j] * (X[lv[j + 1] * D + a] - X[lv[0] * D + a]);
    out[t * D + a] = x;
  }
}

__global__ void k_interp_points_vol(int D, int nq, const double* __restrict__ xr, const double* __restrict__ xyz,
                                    int64_t E, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * nq) return;
  const int64_t e = t / nq;
  const int q = (int)(t - e * nq);
  const double* X = xyz + e * (D + 1) * D;
  for (int a = 0; a < D; ++a) {
    double x = X[a];
    for (int cc = 0; cc < D; ++cc) x += xr[q * D + cc] * (X[(cc + 1) * D + a] - X[a]);
    out[t * D + a] = x;
  }
}

// facet DoF: int (u . n_F) psi_j ds (param measure); n_F the global facet normal
__global__ void k_interp_facet(int D, int nqs, int nf, const double* __restrict__ vals,
                               const double* __restrict__ ws, const double* __restrict__ psi, DevMesh mesh,
                               double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mesh.F * nf) return;
  const int64_t F = t / nf;
  const int j = (int)(t - F * nf);
  const int64_t T = mesh.facet_elem[2 * F];
  const int i = mesh.facet_local[2 * F];
  const double* g = mesh.geo + T * GEO_STRIDE;
  const double sigma = ((i & 1) ? -1.0 : 1.0) * (g[GEO_DET] > 0 ? 1.0 : -1.0);
  double n[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) n[a] = sigma * g[GEO_NRM + i * D + a];
  double s = 0.0;
  for (int q = 0; q < nqs; ++q) {
    double un = 0.0;
    for (int a = 0; a < D; ++a) un += vals[(F * nqs + q) * D + a] * n[a];
    s += ws[q] * un * psi[q * nf + j];
  }
  x[t] = s;
}

// interior DoF: |det|^{-(d-1)/d} int (det J^{-1} u) . q_m dx^
__global__ void k_interp_int(int D, int nq, int nint, const double* __restrict__ vals, const double* __restrict__ w,
                             const double* __restrict__ qm, DevMesh mesh, double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mesh.E * nint) return;
  const int64_t e = t / nint;
  const int mi = (int)(t - e * nint);
  const double* g = mesh.geo + e * GEO_STRIDE;
  double adj[3][3];
  if (D == 2) {
    adj[0][0] = g[3]; adj[0][1] = -g[1]; adj[1][0] = -g[2]; adj[1][1] = g[0];
  } else {
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        const int r1 = (cc + 1) % 3, r2 = (cc + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        adj[r][cc] = g[r1 * 3 + c1] * g[r2 * 3 + c2] - g[r1 * 3 + c2] * g[r2 * 3 + c1];
      }
  }
  double s = 0.0;
  for (int q = 0; q < nq; ++q) {
    const double* u = vals + (e * nq + q) * D;
    for (int a = 0; a < D; ++a) {
      double uh = 0.0;
      for (int b = 0; b < D; ++b) uh += adj[a][b] * u[b];
      s += w[q] * uh * qm[(q * nint + mi) * D + a];
    }
  }
  x[t] = s / g[GEO_SI];
}

// u at reference points: u = J u^ / det, u^ = sum_j x^_j phi^_j
__global__ void k_eval(int D, int n, int nf, int nint, int np, const double* __restrict__ x,
                       const double* __restrict__ phi, DevMesh mesh, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mesh.E * np) return;
  const int64_t e = t / np;
  const int p = (int)(t - e * np);
  const double* g = mesh.geo + e * GEO_STRIDE;
  const int nfl = (D + 1) * nf;
  const int64_t off = mesh.F * nf;
  double uh[3] = {0, 0, 0};
  for (int j = 0; j < n; ++j) {
    double v = 0.0;
    if (j < nfl) {
      const int f = j / nf;
      const int32_t F = mesh.fid[e * (D + 1) + f];
      if (F >= 0) v = x[(int64_t)F * nf + (j - f * nf)] * g[GEO_NFN + f];
    } else {
      v = x[off + e * nint + (j - nfl)] * g[GEO_SI];
    }
    for (int a = 0; a < D; ++a) uh[a] += v * phi[(p * n + j) * D + a];
  }
  for (int a = 0; a < D; ++a) {
    double s = 0;
    for (int b = 0; b < D; ++b) s += g[a * D + b] * uh[b];
    out[t * D + a] = s / g[GEO_DET];
  }
}

// Adaptive HOPU order: eta = num/den per facet and l from the thresholds
// eta_0 < ... < eta_k (eta_{k+1} = 1): eta_i < eta <= eta_{i+1} -> i,
// eta <= eta_0 -> -1, eta > 1 -> k.  den = 0 gives eta = 0 (num = 0) or +inf.
struct Thresholds {
  double t[8];
  int k;
};
__global__ void k_adapt(const double* __restrict__ eta_nd, int64_t F, Thresholds th, int8_t* __restrict__ lfac,
                        double* __restrict__ eta_out) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const double num = eta_nd[2 * f], den = eta_nd[2 * f + 1];
  const double eta = den > 0 ? num / den : (num > 0 ? INFINITY : 0.0);
  if (eta_out) eta_out[f] = eta;
  if (!lfac) return;
  int l = -1;
  for (int i = 0; i <= th.k; ++i) {
    const double hi = i < th.k ? th.t[i + 1] : 1.0;
    if (eta > th.t[i] && eta <= hi) l = i;
  }
  if (eta > 1.0) l = th.k;
  lfac[f] = (int8_t)l;
}

// ------------------------------------------------------------------ launchers
void launch_adapt(hipStream_t s, const double* eta_nd, int64_t F, const double* thr, int k, int8_t* lfac,
                  double* eta_out) {
  Thresholds th;
  for (int i = 0; i < 8; ++i) th.t[i] = i <= k && thr ? thr[i] : 0.0;
  th.k = k;
  if (F > 0)
    hipLaunchKernelGGL(k_adapt, dim3((unsigned)((F + 255) / 256)), dim3(256), 0, s, eta_nd, F, th, lfac, eta_out);
}

template <int D, int KK>
void launch_energy(hipStream_t s, const double* m, const DevMesh& mesh, double* part) {
  hipLaunchKernelGGL((k_energy<D, KK>), dim3(AUX_NPART), dim3(256), 0, s, m, mesh, part);
}
template <int D, int KK>
int64_t launch_div(hipStream_t s, const double* m, const DevMesh& mesh, const double* fdV, const double* wv,
                   double* part) {
  const int64_t nw = (mesh.E + 15) / 16;
  hipLaunchKernelGGL((k_div<D, KK>), dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, m, mesh, fdV, wv, part);
  return nw;
}
void launch_interp_points(hipStream_t s, int D, int nqs, const double* sp, int nqv, const double* xr,
                          const double* xyz, const DevMesh& mesh, double* pf, double* pv) {
  int64_t n1 = mesh.F * nqs, n2 = mesh.E * nqv;
  if (n1 > 0 && pf)
    hipLaunchKernelGGL(k_interp_points_facet, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, D, nqs, sp,
                       xyz, mesh, pf);
  if (n2 > 0 && pv)
    hipLaunchKernelGGL(k_interp_points_vol, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, D, nqv, xr, xyz,
                       mesh.E, pv);
}
void launch_interpolate(hipStream_t s, int D, int nqs, int nf, const double* vf, const double* ws,
                        const double* psi, int nqv, int nint, const double* vv, const double* wv,
                        const double* qm, const DevMesh& mesh, double* x) {
  int64_t n1 = mesh.F * nf, n2 = mesh.E * nint;
  if (n1 > 0)
    hipLaunchKernelGGL(k_interp_facet, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, D, nqs, nf, vf, ws, psi,
                       mesh, x);
  if (n2 > 0)
    hipLaunchKernelGGL(k_interp_int, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, D, nqv, nint, vv, wv, qm,
                       mesh, x + mesh.F * nf);
}
// Number of NaN / infinite entries of v (an integer count: the atomic adds
// commute, so the result is exact and order-independent).
__global__ void k_zero_count(unsigned long long* count) { *count = 0ull; }
__global__ __launch_bounds__(256) void k_count_nonfinite(const double* __restrict__ v, int64_t n,
                                                         unsigned long long* count) {
  unsigned int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    c += isfinite(v[i]) ? 0u : 1u;
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) c += __shfl_xor(c, sh, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}
void launch_count_nonfinite(hipStream_t s, const double* v, int64_t n, unsigned long long* count) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, count);
  const int64_t b = std::min<int64_t>((n + 255) / 256, 2048);
  if (n > 0) hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)b), dim3(256), 0, s, v, n, count);
}

void launch_eval(hipStream_t s, int D, int n, int nf, int nint, int np, const double* x, const double* phi,
                 const DevMesh& mesh, double* out) {
  int64_t nt = mesh.E * np;
  if (nt > 0)
    hipLaunchKernelGGL(k_eval, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, D, n, nf, nint, np, x, phi, mesh,
                       out);
}

#define HOPU_AUX_INST(D, KK)                                                                    \
  template void launch_energy<D, KK>(hipStream_t, const double*, const DevMesh&, double*);      \
  template int64_t launch_div<D, KK>(hipStream_t, const double*, const DevMesh&, const double*, \
                                     const double*, double*);
HOPU_AUX_INST(2, 1)
HOPU_AUX_INST(2, 2)
HOPU_AUX_INST(2, 3)
HOPU_AUX_INST(2, 4)
HOPU_AUX_INST(3, 1)
HOPU_AUX_INST(3, 2)
HOPU_AUX_INST(3, 3)
HOPU_AUX_INST(3, 4)
HOPU_AUX_INST(3, 5)

}  // namespace hopu

namespace hopu {

// Measurement only: sustained FP64 MFMA rate of independent 16x16x4
// accumulation chains held in registers (no memory, no LDS), one block of
// four waves per CU times `blocks_per_cu`.
__global__ __launch_bounds__(256) void k_mfma_f64_rate(double* __restrict__ out, int iters, double a0, double b0) {
  typedef double d4v __attribute__((ext_vector_type(4)));
  d4v acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = d4v{0, 0, 0, 0};
  const double a = a0 + threadIdx.x * 1e-9, b = b0 + blockIdx.x * 1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

void launch_mfma_f64_rate(hipStream_t s, double* out, int blocks, int iters) {
  hipLaunchKernelGGL(k_mfma_f64_rate, dim3((unsigned)blocks), dim3(256), 0, s, out, iters, 1.0, 1e-3);
}

}  // namespace hopu
