// Projection step of the operator splitting (paper section 2.3, eq.
// (MCS_step2)), condensed onto the facet multipliers p^ and solved matrix-free.
//
// Per element, in the modal coordinates of the mass kernels (m = Dinv S x,
// M_T = S Dinv^T (G (x) I) Dinv S / |det|, Z = (G^-1 (x) I) |det| the modal
// inverse mass) and with Bm[beta][rho] = int_T^ d_a p_alpha q_beta the
// reference divergence moments (b1(v, q_beta) = -sgn(det) (Bm m)_beta):
//     A   = Bm Z Bm^t                      (nQ x nQ, SPD; inverted at set-up)
//     t_f = Z D^t S^-1 C^t p^              (C^t p^: sigma_{T,F} p^_F on the
//                                           facet rows, 0 on interior rows)
//     tau = t_f - Z Bm^t A^-1 Bm (t_f - m*)
//     u~_T = S^-1 D tau
// and the multipliers solve  S_p p^ = g  with
//     S_p p^ = sum_T C_T S^-1 D (t_f - Z Bm^t A^-1 Bm t_f)
//     g      = - sum_T C_T S^-1 D Z Bm^t A^-1 Bm m*.
// sigma_{T,F} = (-1)^i sgn(det J) is the outward sign of the facet normal
// N_F for local facet i.  Rows follow the mass kernels' order (lane group g
// holds facet g's rows at steps s < n_f, interior rows elsewhere).
#include "kernels.hpp"
#include "launch_events.hpp"
#include "proj.hpp"

namespace hopu {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {
// modal tiles (register i of tile mt, lane group g: row 16 mt + 4 i + g) and
// per-step values, as array types (a template-id with a comma inside a
// parameter's array bound does not parse)
template <int D, int KK>
using Tiles = double[Cfg<D, KK>::NMT][4];
template <int D, int KK>
using Steps = double[Cfg<D, KK>::NK];

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 d4zero() { d4 v = {0, 0, 0, 0}; return v; }

// the row order of the mass tables (kernels.hip): facet row s of facet g, or
// interior row t
template <int D, int KK>
__device__ __forceinline__ bool is_facet(int s, int g) {
  return s < Cfg<D, KK>::NF && g <= D;
}
template <int D, int KK>
__device__ __forceinline__ int int_row(int s, int g) {
  using C = Cfg<D, KK>;
  constexpr int nfg = D + 1;
  return s < C::NF ? s * (4 - nfg) + (g - nfg) : C::NF * (4 - nfg) + (s - C::NF) * 4 + g;
}

template <int D>
__device__ __forceinline__ void inv_gram_det(const double* Gr, double Gs[D][D]) {
  // G^-1 |det J| = adj(G) / |det J|  (det G = det J^2), G = J^t J
  double J[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) J[r][c] = Gr[r * D + c];
  double Gm[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double s = 0;
#pragma unroll
      for (int r = 0; r < D; ++r) s += J[r][a] * J[r][b];
      Gm[a][b] = s;
    }
  const double sd = 1.0 / fabs(Gr[GEO_DET]);
  if (D == 2) {
    Gs[0][0] = Gm[1][1] * sd; Gs[1][1] = Gm[0][0] * sd;
    Gs[0][1] = -Gm[0][1] * sd; Gs[1][0] = -Gm[1][0] * sd;
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const int a1 = (b + 1) % 3, a2 = (b + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        Gs[a][b] = (Gm[a1][b1] * Gm[a2][b2] - Gm[a1][b2] * Gm[a2][b1]) * sd;
      }
  }
}

// y <- Z y in the modal tile layout (quads blk*D + a hold component a)
template <int D, int KK>
__device__ __forceinline__ void zmix(Tiles<D, KK>& y, const double (&Gs)[D][D]) {
  using C = Cfg<D, KK>;
#pragma unroll
  for (int blk = 0; blk < C::NPK; ++blk) {
    double t[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double s = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const int rq = blk * D + b;
        s += Gs[a][b] * y[rq / 4][rq % 4];
      }
      t[a] = s;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) y[(blk * D + a) / 4][(blk * D + a) % 4] = t[a];
  }
}

// out (modal tiles) = table (NMT tiles x NK steps) . xin (one value per
// step); only the first NKU steps are nonzero
template <int D, int KK, int NKU>
__device__ __forceinline__ void contract_in(const double* __restrict__ tab, const Steps<D, KK>& xin,
                                            Tiles<D, KK>& y, int lane) {
  using C = Cfg<D, KK>;
#pragma unroll
  for (int mt = 0; mt < C::NMT; ++mt) {
    d4 acc = d4zero();
#pragma unroll
    for (int kk = 0; kk < NKU; ++kk) acc = mfma(tab[(mt * C::NK + kk) * 64 + lane], xin[kk], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) y[mt][i] = acc[i];
  }
}

// tau <- tau - Z Bm^t A^-1 Bm v  (v in modal tiles); A^-1 of element e
template <int D, int KK>
__device__ __forceinline__ void schur_correct(const Tiles<D, KK>& v, Tiles<D, KK>& tau, const double (&Gs)[D][D],
                                              const ProjDev& pj, int64_t ee, int lane) {
  using C = Cfg<D, KK>;
  constexpr int NQ = C::NQ, NBT = (NQ + 15) / 16, NQK = (NQ + 3) / 4;
  const int g = lane >> 4, c = lane & 15;
  // r = Bm v: tile bt, register i of group g holds beta = 16 bt + 4 i + g
  double r[NBT][4];
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt) {
    d4 acc = d4zero();
#pragma unroll
    for (int rq = 0; rq < C::NMQ; ++rq) acc = mfma(pj.b[(bt * C::NMQ + rq) * 64 + lane], v[rq / 4][rq % 4], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) r[bt][i] = acc[i];
  }
  // y = A^-1 r: every lane gathers its element's r by shuffles
  double y[NBT][4];
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt)
#pragma unroll
    for (int i = 0; i < 4; ++i) y[bt][i] = 0.0;
  const double* Ai = pj.ainv + ee * NQ * NQ;
#pragma unroll
  for (int ga = 0; ga < NQ; ++ga) {
    const double rg = __shfl(r[ga / 16][(ga % 16) / 4], 16 * (ga % 4) + c, 64);
#pragma unroll
    for (int bt = 0; bt < NBT; ++bt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int be = 16 * bt + 4 * i + g;
        if (be < NQ) y[bt][i] += Ai[be * NQ + ga] * rg;
      }
  }
  // w = Bm^t y (modal tiles), then tau -= Z w
  double w[C::NMT][4];
#pragma unroll
  for (int mt = 0; mt < C::NMT; ++mt) {
    d4 acc = d4zero();
#pragma unroll
    for (int kk = 0; kk < NQK; ++kk) acc = mfma(pj.bt[(mt * NQK + kk) * 64 + lane], y[kk / 4][kk % 4], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) w[mt][i] = acc[i];
  }
  zmix<D, KK>(w, Gs);
#pragma unroll
  for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) tau[mt][i] -= w[mt][i];
}
}  // namespace

// MODE 0: facet-side contributions of S_p p^ (+ per-block p^ . S_p p^)
// MODE 1: facet-side contributions of g (from u*)
// MODE 2: u_new = u* - u~ (from p^ and u*), rows written once
template <int D, int KK, int MODE>
__global__ __launch_bounds__(256) void k_proj(const double* __restrict__ ph, const double* __restrict__ us,
                                              double* __restrict__ out, DevMesh mesh, ProjDev pj,
                                              double* __restrict__ part, const int* __restrict__ flag) {
  using C = Cfg<D, KK>;
  if (flag && *flag) return;  // CG converged: iterations queued after it do nothing
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t e = wave * 16 + c;
  const bool valid = e < mesh.E;
  const int64_t ee = valid ? e : 0;
  const double* Gr = mesh.geo + ee * GEO_STRIDE;
  const int gg = g <= D ? g : D;
  const bool fl = valid && g <= D;                   // this lane's facet exists
  const int32_t mf = fl ? pj.mfid[ee * (D + 1) + gg] : -1;   // multiplier block
  const int32_t fid = fl ? mesh.fid[ee * (D + 1) + gg] : -1; // V_h facet (-1: wall)
  const int side = (fid >= 0) ? (int)mesh.fside[ee * (D + 1) + gg] : 0;
  const double det = Gr[GEO_DET];
  const double sig = ((gg % 2) ? -1.0 : 1.0) * (det > 0 ? 1.0 : -1.0);
  const double nf = Gr[GEO_NFN + gg];
  const double si = Gr[GEO_SI];
  const int64_t off = mesh.F * C::NF;
  double Gs[D][D];
  inv_gram_det<D>(Gr, Gs);

  double tau[C::NMT][4], w1[C::NMT][4];
  if (MODE != 1) {
    // t_f = Z D^t S^-1 C^t p^
    double f[C::NK];
#pragma unroll
    for (int kk = 0; kk < C::NK; ++kk)
      f[kk] = (is_facet<D, KK>(kk, g) && mf >= 0) ? sig * ph[(int64_t)mf * C::NF + kk] / nf : 0.0;
    // (f vanishes on the interior steps s >= n_f)
    contract_in<D, KK, C::NF>(pj.prec_in, f, w1, lane);
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) tau[mt][i] = w1[mt][i];
    zmix<D, KK>(tau, Gs);
  } else {
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) tau[mt][i] = 0.0;
  }
  double xs[C::NK];
  double v[C::NMT][4];
  if (MODE != 0) {
    // m* = Dinv S u*
#pragma unroll
    for (int kk = 0; kk < C::NK; ++kk) {
      double x = 0.0;
      if (valid) {
        if (is_facet<D, KK>(kk, g)) {
          if (fid >= 0) x = us[(int64_t)fid * C::NF + kk];
        } else {
          const int t = int_row<D, KK>(kk, g);
          if (t < C::NINT) x = us[off + ee * C::NINT + t];
        }
      }
      xs[kk] = x;
    }
    double xh[C::NK];
#pragma unroll
    for (int kk = 0; kk < C::NK; ++kk) xh[kk] = xs[kk] * (is_facet<D, KK>(kk, g) ? nf : si);
    double ms[C::NMT][4];
    contract_in<D, KK, C::NK>(pj.mass_in, xh, ms, lane);
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[mt][i] = tau[mt][i] - ms[mt][i];
  } else {
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[mt][i] = tau[mt][i];
  }
  // tau = t_f - Z Bm^t A^-1 Bm (t_f - m*)
  schur_correct<D, KK>(v, tau, Gs, pj, ee, lane);

  double dot = 0.0;
  if (MODE == 0) {
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) dot += w1[mt][i] * tau[mt][i];
  }
  // u~ rows = S^-1 D tau (output tile jt, register i = step 4 jt + i); modes
  // 0 and 1 need the facet steps s < n_f only
  constexpr int NJO = MODE == 2 ? C::NJT : (C::NF + 3) / 4;
#pragma unroll
  for (int jt = 0; jt < NJO; ++jt) {
    d4 o = d4zero();
#pragma unroll
    for (int rq = 0; rq < C::NMQ; ++rq) o = mfma(pj.prec_out[(jt * C::NMQ + rq) * 64 + lane], tau[rq / 4][rq % 4], o);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = 4 * jt + i;
      if (s >= C::NK || !valid) continue;
      if (is_facet<D, KK>(s, g)) {
        const double ut = o[i] / nf;
        if (MODE != 2) {
          // S_p p^ (mode 0) is + C_T u~ of the p^-part; g (mode 1) is - C_T of
          // the u*-part, which tau holds here
          if (mf >= 0) out[((int64_t)side * pj.FW + mf) * C::NF + s] = (MODE == 0 ? sig : -sig) * ut;
        } else if (fid >= 0 && side == 0) {
          out[(int64_t)fid * C::NF + s] = xs[s] - ut;
        }
      } else if (MODE == 2) {
        const int t = int_row<D, KK>(s, g);
        if (t < C::NINT) out[off + e * C::NINT + t] = xs[s] - o[i] / si;
      }
    }
  }
  if (MODE == 0 && part) {
    __shared__ double red[4];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) dot += __shfl_xor(dot, s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// A^-1 = (Bm Z Bm^t)^-1 per element: one thread per element, in place in
// the output (Gauss-Jordan; A is SPD, no pivoting needed)
template <int D, int KK>
__global__ void k_proj_ainv(DevMesh mesh, const double* __restrict__ kab, double* __restrict__ ainv) {
  using C = Cfg<D, KK>;
  constexpr int NQ = C::NQ;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mesh.E) return;
  double Gs[D][D];
  inv_gram_det<D>(mesh.geo + e * GEO_STRIDE, Gs);
  double* A = ainv + e * NQ * NQ;
  for (int i = 0; i < NQ * NQ; ++i) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) s += Gs[a][b] * kab[(a * D + b) * NQ * NQ + i];
    A[i] = s;
  }
  for (int k = 0; k < NQ; ++k) {
    const double piv = 1.0 / A[k * NQ + k];
    A[k * NQ + k] = 1.0;
    for (int j = 0; j < NQ; ++j) A[k * NQ + j] *= piv;
    for (int i = 0; i < NQ; ++i) {
      if (i == k) continue;
      const double f = A[i * NQ + k];
      A[i * NQ + k] = 0.0;
      for (int j = 0; j < NQ; ++j) A[i * NQ + j] -= f * A[k * NQ + j];
    }
  }
}

template <int D, int KK>
int launch_proj(hipStream_t s, int mode, const double* ph, const double* us, double* out, const DevMesh& mesh,
                const ProjDev& pj, double* part, const int* flag) {
  const int64_t waves = (mesh.E + 15) / 16;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0) return 0;
  if (mode == 0)
    HOPU_LAUNCH((k_proj<D, KK, 0>), dim3((unsigned)blocks), dim3(256), 0, s, ph, us, out, mesh, pj, part, flag);
  else if (mode == 1)
    HOPU_LAUNCH((k_proj<D, KK, 1>), dim3((unsigned)blocks), dim3(256), 0, s, ph, us, out, mesh, pj, part, flag);
  else
    HOPU_LAUNCH((k_proj<D, KK, 2>), dim3((unsigned)blocks), dim3(256), 0, s, ph, us, out, mesh, pj, part, flag);
  return (int)blocks;
}

template <int D, int KK>
void launch_proj_ainv(hipStream_t s, const DevMesh& mesh, const double* kab, double* ainv) {
  if (mesh.E == 0) return;
  hipLaunchKernelGGL((k_proj_ainv<D, KK>), dim3((unsigned)((mesh.E + 127) / 128)), dim3(128), 0, s, mesh, kab,
                     ainv);
}

#define HOPU_PROJ_INST(D, KK)                                                                              \
  template int launch_proj<D, KK>(hipStream_t, int, const double*, const double*, double*, const DevMesh&, \
                                  const ProjDev&, double*, const int*);                                    \
  template void launch_proj_ainv<D, KK>(hipStream_t, const DevMesh&, const double*, double*);

HOPU_PROJ_INST(2, 1)
HOPU_PROJ_INST(2, 2)
HOPU_PROJ_INST(2, 3)
HOPU_PROJ_INST(2, 4)
HOPU_PROJ_INST(3, 1)
HOPU_PROJ_INST(3, 2)
HOPU_PROJ_INST(3, 3)
HOPU_PROJ_INST(3, 4)
HOPU_PROJ_INST(3, 5)

}  // namespace hopu
