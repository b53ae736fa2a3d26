// HIP kernels for gfx950.  See kernels.hpp for the batch/tile conventions.
#include <algorithm>
#include <type_traits>

#include "bf16split.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "launch_events.hpp"

namespace hopu {

// Persistent mass kernels: one block of MASS_WPB waves per CU (two waves
// per SIMD), so the tables are copied to LDS once per CU and every CU keeps
// its waves for the whole launch.
static constexpr int MASS_WPB = 8;
static constexpr int64_t MASS_BLOCKS = 256;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
template <> struct MF<double> {
  typedef d4 V;
  // v_mfma_f64_16x16x4f64: row 4i+g of the 16x16 output sits in register i
  // of lane group g.
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int g) { return 4 * i + g; }
};
template <> struct MF<float> {
  typedef f4 V;
  // v_mfma_f32_16x16x4f32: row 4g+i sits in register i of lane group g.
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int g) { return 4 * g + i; }
};

template <typename V> __device__ __forceinline__ V vzero() { V v = {0, 0, 0, 0}; return v; }


// Batches are assigned so that consecutive batches land on the same XCD
// (workgroups are dealt round-robin over the 8 XCDs).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t per = (nblocks + 7) / 8;
  int64_t x = bid % 8, s = bid / 8;
  int64_t full = nblocks % 8 == 0 ? 8 : nblocks % 8;  // XCDs that get `per` blocks
  if (x < full) return x * per + s;
  return full * per + (x - full) * (per - 1) + s;
}

template <int D>
__device__ __forceinline__ void load_J(const double* g, double J[D][D]) {
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) J[r][c] = g[r * D + c];
}

// ------------------------------------------------------------------ modal
// m_T = Dinv (S_T x_T): dual coefficients -> modal coefficients (rho layout),
// stored as TS.  The contraction is FP64 in every precision form: the dual
// basis' condition number grows quickly with k (about 4e5 at k = 5 in 3D),
// so a reduced-precision transform would lose far more than the
// contractions that follow it.
template <typename TS, int D, int KK>
__global__ __launch_bounds__(256) void k_modal(const double* __restrict__ x, TS* __restrict__ m,
                                               DevMesh mesh, const double* __restrict__ frag) {
  using C = Cfg<D, KK>;
  using M = MF<double>;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t e = wave * 16 + c;
  if (wave * 16 >= mesh.E) return;
  const bool valid = e < mesh.E;
  const int64_t ee = valid ? e : 0;
  const double* G = mesh.geo + ee * GEO_STRIDE;
  const int64_t off = mesh.F * C::NF;
  double xh[C::NK];
#pragma unroll
  for (int kk = 0; kk < C::NK; ++kk) {
    const int j = 4 * kk + g;
    double v = 0.0;
    if (valid && j < C::N) {
      if (j < C::NFL) {
        const int f = j / C::NF, jj = j - f * C::NF;
        const int32_t F = mesh.fid[ee * (D + 1) + f];
        if (F >= 0) v = x[(int64_t)F * C::NF + jj] * G[GEO_NFN + f];
      } else {
        v = x[off + ee * C::NINT + (j - C::NFL)] * G[GEO_SI];
      }
    }
    xh[kk] = v;
  }
#pragma unroll
  for (int mt = 0; mt < C::NMT; ++mt) {
    d4 acc = vzero<d4>();
#pragma unroll
    for (int kk = 0; kk < C::NK; ++kk) acc = M::mma(frag[(mt * C::NK + kk) * 64 + lane], xh[kk], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * mt + M::row(i, g);
      if (valid && row < C::NM) m[ee * C::NM + row] = (TS)acc[i];
    }
  }
}

// Residual accumulators of the element kernel.  FP64: the MFMA accumulators
// themselves.  FP32: FP32 MFMA accumulation inside one tile (a quadrature
// tile or one facet's test), added into FP64 across tiles.
template <typename T, int D, int NAT> struct ElemAcc;
template <int D, int NAT> struct ElemAcc<double, D, NAT> {
  d4 v[D][NAT];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < NAT; ++at) v[a][at] = vzero<d4>();
  }
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ d4& tile(int a, int at) { return v[a][at]; }
  __device__ __forceinline__ void end() {}
  __device__ __forceinline__ double get(int a, int at, int i) const { return v[a][at][i]; }
};
template <int D, int NAT> struct ElemAcc<float, D, NAT> {
  double v[D][NAT][4];
  f4 t[D][NAT];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < NAT; ++at)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[a][at][i] = 0.0;
  }
  __device__ __forceinline__ void begin() {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < NAT; ++at) t[a][at] = vzero<f4>();
  }
  __device__ __forceinline__ f4& tile(int a, int at) { return t[a][at]; }
  __device__ __forceinline__ void end() {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < NAT; ++at)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[a][at][i] += (double)t[a][at][i];
  }
  __device__ __forceinline__ double get(int a, int at, int i) const { return v[a][at][i]; }
};

// ------------------------------------------------------------------ element
// Fused convection residual of a batch of 16 elements:
//   volume  - int (u x u) : grad phi, in reference form
//           - sgn(det)/det^2 int (G u^) . (grad^ phi^) u^,  G = J^T J
//   facets  + int (u.n)<u>.phi + (I - Pi)(1/2|u.n|(I - Pi)[[u]]) . phi
//           with [[.]] = own - neighbour and n the own outward normal;
// then r^ = S Dinv^T r_modal.  Facet rows go to per-element slots, interior
// rows straight to r.
// NS > 0 (T = float): the contractions in split BF16 (see mma_bf).
// One wave (one batch) per block: the kernel holds one wave per SIMD, and a
// block of one wave frees its SIMD as soon as it ends (with four-wave
// blocks a SIMD waited for its block's slowest wave; FP64 1.26 -> 1.16 ms).
template <typename T, int D, int KK, int NS = 0>
__global__ __launch_bounds__(64) void k_elem(const T* __restrict__ m, double* __restrict__ r,
                                              double* __restrict__ rslot, DevMesh mesh,
                                              DevTables<TabT<T, NS>> tb, int terms,
                                              double* __restrict__ diss_part, double* __restrict__ eta_nd) {
  using C = Cfg<D, KK>;
  using M = MF<T>;
  using V = typename M::V;
  // the jump indicator of the adaptive order is always evaluated in FP64;
  // the FP32 kernel carries no code for it
  constexpr bool ETA = sizeof(T) == sizeof(double);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t b = xcd_remap(blockIdx.x, mesh.nb);
  if (b >= mesh.nb) return;
  const int32_t e = mesh.belem[b * 16 + c];
  const bool valid = e >= 0;
  const int64_t ee = valid ? e : mesh.belem[b * 16];
  const int sig = mesh.bsig[b];
  const double* Gr = mesh.geo + ee * GEO_STRIDE;
  double J[D][D];
  load_J<D>(Gr, J);
  const double det = Gr[GEO_DET];
  const double idet = 1.0 / det;

  T mB[D][C::NPK];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int kk = 0; kk < C::NPK; ++kk) mB[a][kk] = m[ee * C::NM + kk * 4 * D + 4 * a + g];
  // split-BF16 form: the modal coefficients split once, in groups of four steps
  constexpr int NGP = (C::NPK + 3) / 4;
  BfTab<NS> mS[D][NGP];
  if constexpr (NS > 0) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int sg = 0; sg < NGP; ++sg) mS[a][sg] = bf_steps<NS>(mB[a], 4 * sg);
  }

  ElemAcc<T, D, C::NAT> acc;
  acc.init();

  // ---------------- volume term
  if (terms & 1) {
    double Gm[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        double s = 0;
#pragma unroll
        for (int r2 = 0; r2 < D; ++r2) s += J[r2][a] * J[r2][bb];
        Gm[a][bb] = s;
      }
    const double sc = -idet * idet * (det > 0 ? 1.0 : -1.0);
#pragma unroll 1
    for (int qt = 0; qt < C::NQVT; ++qt) {
      V u[D];
#pragma unroll
      for (int a = 0; a < D; ++a) u[a] = vzero<V>();
      if constexpr (NS == 0) {
#pragma unroll
        for (int kk = 0; kk < C::NPK; ++kk) {
          const T av = tb.vol_V[(qt * C::NPK + kk) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) u[a] = M::mma(av, mB[a][kk], u[a]);
        }
      } else {
#pragma unroll
        for (int sg = 0; sg < NGP; ++sg) {
          const BfTab<NS> av = tb.vol_V[(qt * NGP + sg) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) u[a] = mma_bf<NS>(av, mS[a][sg], u[a]);
        }
      }
      // flux F_ab = w sgn/det^2 (G u^)_a u^_b formed per MFMA operand
      double uh[D][4], gu[D][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 16 * qt + M::row(i, g);
        const double wq = q < C::NQV ? tb.wv[q] : 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) uh[a][i] = (double)u[a][i];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = 0;
#pragma unroll
          for (int bb = 0; bb < D; ++bb) s += Gm[a][bb] * (double)u[bb][i];
          gu[a][i] = s * wq * sc;
        }
      }
      acc.begin();
      if constexpr (NS == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int bb = 0; bb < D; ++bb)
#pragma unroll
            for (int at = 0; at < C::NAT; ++at) {
              const T av = tb.vol_dVT[(((qt * 4 + i) * D + bb) * C::NAT + at) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) acc.tile(a, at) = M::mma(av, (T)(gu[a][i] * uh[bb][i]), acc.tile(a, at));
            }
      } else {
        // the four points i of the tile are one step group
#pragma unroll
        for (int bb = 0; bb < D; ++bb) {
          BfTab<NS> fb[D];
#pragma unroll
          for (int a = 0; a < D; ++a)
            fb[a] = bf_split4<NS>((float)(gu[a][0] * uh[bb][0]), (float)(gu[a][1] * uh[bb][1]),
                                  (float)(gu[a][2] * uh[bb][2]), (float)(gu[a][3] * uh[bb][3]));
#pragma unroll
          for (int at = 0; at < C::NAT; ++at) {
            const BfTab<NS> av = tb.vol_dVT[((qt * D + bb) * C::NAT + at) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) acc.tile(a, at) = mma_bf<NS>(av, fb[a], acc.tile(a, at));
          }
        }
      }
      acc.end();
    }
  }

  // ---------------- facet terms
  double diss = 0.0;
  const bool cen = terms & 2, up = terms & 4;
  if (cen || up) {
#pragma unroll 1
    for (int f = 0; f <= D; ++f) {
      const int fp = (sig >> (4 * f)) & 0xF;
      if (fp == 0xF) continue;  // wall facet for the whole batch: u.n = 0
      const int32_t en = valid ? mesh.nbr[ee * (D + 1) + f] : (int32_t)ee;
      const double* Gn = mesh.geo + (int64_t)en * GEO_STRIDE;
      double Jn[D][D];
      load_J<D>(Gn, Jn);
      const double idetn = 1.0 / Gn[GEO_DET];
      const double nfn = Gr[GEO_NFN + f];
      double nrm[D];
#pragma unroll
      for (int a = 0; a < D; ++a) nrm[a] = Gr[GEO_NRM + f * D + a];
      int lf = mesh.lglob;
      if (mesh.lfac) lf = valid ? (int)mesh.lfac[mesh.fid[ee * (D + 1) + f]] : -1;
      T nB[D][C::NPK];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int kk = 0; kk < C::NPK; ++kk) nB[a][kk] = m[(int64_t)en * C::NM + kk * 4 * D + 4 * a + g];
      BfTab<NS> nS[D][NGP];
      if constexpr (NS > 0) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int sg = 0; sg < NGP; ++sg) nS[a][sg] = bf_steps<NS>(nB[a], 4 * sg);
      }

      // moments of the physical jump against psi_j (deg psi_j <= l)
      T c1[D][C::NFJT][4];
      if (up) {
#pragma unroll
        for (int jt = 0; jt < C::NFJT; ++jt) {
          V ro[D], rn[D];
#pragma unroll
          for (int a = 0; a < D; ++a) { ro[a] = vzero<V>(); rn[a] = vzero<V>(); }
          if constexpr (NS == 0) {
#pragma unroll
            for (int kk = 0; kk < C::NPK; ++kk) {
              const T ao = tb.fac_K[((f * C::NFJT + jt) * C::NPK + kk) * 64 + lane];
              const T an = tb.fac_K[((fp * C::NFJT + jt) * C::NPK + kk) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) {
                ro[a] = M::mma(ao, mB[a][kk], ro[a]);
                rn[a] = M::mma(an, nB[a][kk], rn[a]);
              }
            }
          } else {
#pragma unroll
            for (int sg = 0; sg < NGP; ++sg) {
              const BfTab<NS> ao = tb.fac_K[((f * C::NFJT + jt) * NGP + sg) * 64 + lane];
              const BfTab<NS> an = tb.fac_K[((fp * C::NFJT + jt) * NGP + sg) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) {
                ro[a] = mma_bf<NS>(ao, mS[a][sg], ro[a]);
                rn[a] = mma_bf<NS>(an, nS[a][sg], rn[a]);
              }
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int j = 16 * jt + M::row(i, g);
            const bool keep = j < C::NF && tb.psi_deg[j < C::NF ? j : 0] <= lf;
#pragma unroll
            for (int a = 0; a < D; ++a) {
              double s = 0;
#pragma unroll
              for (int bb = 0; bb < D; ++bb)
                s += J[a][bb] * (double)ro[bb][i] * idet - Jn[a][bb] * (double)rn[bb][i] * idetn;
              c1[a][jt][i] = keep ? (T)s : (T)0;
            }
          }
        }
      }
      V c2[D][C::NFJT];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int jt = 0; jt < C::NFJT; ++jt) c2[a][jt] = vzero<V>();
      double eta_num = 0.0, eta_den = 0.0;  // jump indicator of the adaptive order

#pragma unroll 1
      for (int qt = 0; qt < C::NQFT; ++qt) {
        V to[D], tn[D], pj[D];
#pragma unroll
        for (int a = 0; a < D; ++a) { to[a] = vzero<V>(); tn[a] = vzero<V>(); pj[a] = vzero<V>(); }
        if constexpr (NS == 0) {
#pragma unroll
          for (int kk = 0; kk < C::NPK; ++kk) {
            const T ao = tb.fac_Tr[((f * C::NQFT + qt) * C::NPK + kk) * 64 + lane];
            const T an = tb.fac_Tr[((fp * C::NQFT + qt) * C::NPK + kk) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) {
              to[a] = M::mma(ao, mB[a][kk], to[a]);
              tn[a] = M::mma(an, nB[a][kk], tn[a]);
            }
          }
          if (up) {
#pragma unroll
            for (int jk = 0; jk < C::NFK; ++jk) {
              const T ap = tb.fac_Psi[(qt * C::NFK + jk) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) pj[a] = M::mma(ap, c1[a][jk / 4][jk % 4], pj[a]);
            }
          }
        } else {
#pragma unroll
          for (int sg = 0; sg < NGP; ++sg) {
            const BfTab<NS> ao = tb.fac_Tr[((f * C::NQFT + qt) * NGP + sg) * 64 + lane];
            const BfTab<NS> an = tb.fac_Tr[((fp * C::NQFT + qt) * NGP + sg) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) {
              to[a] = mma_bf<NS>(ao, mS[a][sg], to[a]);
              tn[a] = mma_bf<NS>(an, nS[a][sg], tn[a]);
            }
          }
          if (up) {
            // steps jk = 4 jt + i of the moments: group jt holds c1[.][jt][0..3]
#pragma unroll
            for (int jt = 0; jt < C::NFJT; ++jt) {
              const BfTab<NS> ap = tb.fac_Psi[(qt * C::NFJT + jt) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a)
                pj[a] = mma_bf<NS>(ap, bf_split4<NS>(c1[a][jt][0], c1[a][jt][1], c1[a][jt][2], c1[a][jt][3]), pj[a]);
            }
          }
        }
        T h[D][4], aw[D][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = 16 * qt + M::row(i, g);
          const double wq = q < C::NQF ? tb.wf[q] : 0.0;
          double uo[D], un[D], avg[D], jp[D];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            double so = 0, sn = 0;
#pragma unroll
            for (int bb = 0; bb < D; ++bb) { so += J[a][bb] * (double)to[bb][i]; sn += Jn[a][bb] * (double)tn[bb][i]; }
            uo[a] = so * idet;
            un[a] = sn * idetn;
          }
          double unn = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) { avg[a] = 0.5 * (uo[a] + un[a]); unn += avg[a] * nrm[a]; }
          const double hu = 0.5 * fabs(unn);
          double gg[D], jj2 = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            jp[a] = (uo[a] - un[a]) - (double)pj[a][i];
            const double av_ = up ? hu * jp[a] : 0.0;
            gg[a] = (cen ? unn * avg[a] : 0.0) + av_;
            aw[a][i] = (T)av_;
            jj2 += jp[a] * jp[a];
          }
          if (up && valid) diss += 0.5 * wq * nfn * hu * jj2;
          if (ETA && eta_nd) {
            double aa = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) aa += avg[a] * avg[a];
            eta_num += wq * nfn * sqrt(jj2);
            eta_den += wq * nfn * sqrt(aa);
          }
          const double sh = wq * nfn * idet;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            double s = 0;
#pragma unroll
            for (int bb = 0; bb < D; ++bb) s += J[bb][a] * gg[bb];
            h[a][i] = (T)(s * sh);
          }
        }
        acc.begin();
        if constexpr (NS == 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int at = 0; at < C::NAT; ++at) {
              const T av = tb.fac_TrT[(((f * C::NQFT + qt) * 4 + i) * C::NAT + at) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) acc.tile(a, at) = M::mma(av, h[a][i], acc.tile(a, at));
            }
        } else {
          BfTab<NS> hb[D];
#pragma unroll
          for (int a = 0; a < D; ++a) hb[a] = bf_split4<NS>(h[a][0], h[a][1], h[a][2], h[a][3]);
#pragma unroll
          for (int at = 0; at < C::NAT; ++at) {
            const BfTab<NS> av = tb.fac_TrT[((f * C::NQFT + qt) * C::NAT + at) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) acc.tile(a, at) = mma_bf<NS>(av, hb[a], acc.tile(a, at));
          }
        }
        acc.end();
        if (up) {
          if constexpr (NS == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int jt = 0; jt < C::NFJT; ++jt) {
                const T ap = tb.fac_PsiT[((qt * 4 + i) * C::NFJT + jt) * 64 + lane];
#pragma unroll
                for (int a = 0; a < D; ++a) c2[a][jt] = M::mma(ap, aw[a][i], c2[a][jt]);
              }
          } else {
            BfTab<NS> ab[D];
#pragma unroll
            for (int a = 0; a < D; ++a) ab[a] = bf_split4<NS>(aw[a][0], aw[a][1], aw[a][2], aw[a][3]);
#pragma unroll
            for (int jt = 0; jt < C::NFJT; ++jt) {
              const BfTab<NS> ap = tb.fac_PsiT[(qt * C::NFJT + jt) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) c2[a][jt] = mma_bf<NS>(ap, ab[a], c2[a][jt]);
            }
          }
        }
      }
      if (ETA && eta_nd) {
        // sum over the four lane groups holding this element's points; the
        // lower element id of the facet writes
        eta_num += __shfl_xor(eta_num, 16, 64);
        eta_num += __shfl_xor(eta_num, 32, 64);
        eta_den += __shfl_xor(eta_den, 16, 64);
        eta_den += __shfl_xor(eta_den, 32, 64);
        if (valid && g == 0 && en > (int32_t)ee) {
          const int64_t F = mesh.fid[ee * (D + 1) + f];
          eta_nd[2 * F] = eta_num;
          eta_nd[2 * F + 1] = eta_den;
        }
      }
      if (up) {
        // subtract the test of Pi(a): sum_j K_f[j][alpha] |N_F| (J^T c2_j)/det
        T cc[D][C::NFJT][4];
#pragma unroll
        for (int jt = 0; jt < C::NFJT; ++jt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int j = 16 * jt + M::row(i, g);
            const bool keep = j < C::NF && tb.psi_deg[j < C::NF ? j : 0] <= lf;
#pragma unroll
            for (int a = 0; a < D; ++a) {
              double s = 0;
#pragma unroll
              for (int bb = 0; bb < D; ++bb) s += J[bb][a] * (double)c2[bb][jt][i];
              cc[a][jt][i] = keep ? (T)(-s * nfn * idet) : (T)0;
            }
          }
        acc.begin();
        if constexpr (NS == 0) {
#pragma unroll
          for (int jk = 0; jk < C::NFK; ++jk)
#pragma unroll
            for (int at = 0; at < C::NAT; ++at) {
              const T av = tb.fac_KT[((f * C::NAT + at) * C::NFK + jk) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) acc.tile(a, at) = M::mma(av, cc[a][jk / 4][jk % 4], acc.tile(a, at));
            }
        } else {
#pragma unroll
          for (int jt = 0; jt < C::NFJT; ++jt) {
            BfTab<NS> cb[D];
#pragma unroll
            for (int a = 0; a < D; ++a) cb[a] = bf_split4<NS>(cc[a][jt][0], cc[a][jt][1], cc[a][jt][2], cc[a][jt][3]);
#pragma unroll
            for (int at = 0; at < C::NAT; ++at) {
              const BfTab<NS> av = tb.fac_KT[((f * C::NAT + at) * C::NFJT + jt) * 64 + lane];
#pragma unroll
              for (int a = 0; a < D; ++a) acc.tile(a, at) = mma_bf<NS>(av, cb[a], acc.tile(a, at));
            }
          }
        }
        acc.end();
      }
    }
  }

  // ---------------- dual transform and write-out, in FP64 for every form
  // (the conditioning of the dual basis; see k_modal), from the FP64 sums
  // across tiles.  The reduced forms' table has the FP64 values with their
  // own K order (modal row 4g + i at register i of lane group g).
  const int64_t off = mesh.F * C::NF;
  const double* const dual = dual_f64(tb);
#pragma unroll
  for (int jt = 0; jt < C::NJT; ++jt) {
    d4 o = vzero<d4>();
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < C::NAT; ++at)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          o = MF<double>::mma(dual[((((jt * D + a) * C::NAT + at) * 4) + i) * 64 + lane], acc.get(a, at, i), o);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = 16 * jt + MF<double>::row(i, g);
      if (valid && j < C::N) {
        if (j < C::NFL) rslot[ee * C::NFL + j] = (double)o[i] * Gr[GEO_NFN + j / C::NF];
        else r[off + ee * C::NINT + (j - C::NFL)] = (double)o[i] * Gr[GEO_SI];
      }
    }
  }
  if (diss_part) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) diss += __shfl_xor(diss, s, 64);
    if (lane == 0) diss_part[b] = diss;
  }
}

// ------------------------------------------------------------------ mass
// MODE 0: y = M_T x_T  = S Dinv^T (G (x) I) Dinv S x_T / |det J|
// MODE 1: y = (M_T^-1)(1/2 facet rows)  = 1/2 S^-1 D (G^-1 (x) I) D^T S^-1 (1/2) x_T |det J|
// Interior rows go to out.  Facet rows go to the facet-side buffer fs, laid
// out [side][F][NF]: each interior facet receives exactly one contribution
// per side, and the assembled row is fs[0][F] + fs[1][F], added by whichever
// kernel consumes it.  Since y = sum_T R_T y_T, the inner product x . y is
// the sum over elements of x_T . y_T, which each lane accumulates locally.
// Each wave walks batches of 16 elements with a grid stride and gathers the
// next batch while the MFMAs of the current one run.
// A lane's per-batch inputs come in two stages, each issued one batch ahead
// of its use, so that no global load is waited on between the MFMAs of a
// batch: the facet ids and sides of element c (needed to address the
// gather), then the gathered rows and the element's geometry.  The hardware
// retires vector-memory loads in order, so a load issued inside the compute
// phase would also wait for every prefetch issued before it.
// Table fragments are read MASS_PF steps ahead of the MFMAs that use them;
// the fences keep the scheduler from moving the reads back down to their
// uses (which would expose the LDS latency at every step).
#ifndef MASS_PF
#define MASS_PF 2
#endif
#define MASS_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

// Row order of the mass kernels (the tables follow it): at step s, lane
// group g holds row s of facet g while s < NF and g <= d; every other slot,
// taken in (s, g) order, holds the next interior row.  A lane therefore
// touches a single facet, whose id, side and scale it keeps in scalars.
template <int D, int KK>
__device__ __forceinline__ bool mass_is_facet(int s, int g) {
  return s < Cfg<D, KK>::NF && g <= D;
}
template <int D, int KK>
__device__ __forceinline__ int mass_int_row(int s, int g) {
  using C = Cfg<D, KK>;
  constexpr int nfg = D + 1;
  return s < C::NF ? s * (4 - nfg) + (g - nfg) : C::NF * (4 - nfg) + (s - C::NF) * 4 + g;
}

// A lane's per-batch inputs come in two stages, each issued one batch ahead
// of its use, so that no global load is waited on between the MFMAs of a
// batch: the id and side of the lane's facet (needed to address the
// gather), then the gathered rows and the element's geometry.  The hardware
// retires vector-memory loads in order, so a load issued inside the compute
// phase would also wait for every prefetch issued before it.
struct MassIdx {
  int32_t fid;   // global facet id of facet g, -1 for none (wall, padding, g > d)
  int32_t side;  // 0/1: which contribution of that facet this element writes
};
template <int D, int KK>
struct MassData {
  double x[Cfg<D, KK>::NK];  // rows held at steps kk, unscaled
  double J[D][D];
  double det, si, nf;  // det J, interior scale, |N_F| of facet g
  MassIdx ix;          // the facet these rows came from (for the output)
};

// All loads below are unconditional (indices clamped into range; what is
// invalid is masked where the values are used): a load under a branch
// makes the compiler merge its result right away, which waits for it.
template <int D>
__device__ __forceinline__ void mass_load_idx(const DevMesh& mesh, int64_t wave, int g, int c, MassIdx& ix) {
  const int64_t e = wave * 16 + c;
  const int64_t ee = e < mesh.E ? e : 0;
  const int gg = g <= D ? g : D;
  ix.fid = mesh.fid[ee * (D + 1) + gg];
  ix.side = (int32_t)mesh.fside[ee * (D + 1) + gg];
}

template <int D, int KK>
__device__ __forceinline__ void mass_load_data(const double* __restrict__ x, const DevMesh& mesh, int64_t wave,
                                               int g, int c, const MassIdx& ix, MassData<D, KK>& md) {
  using C = Cfg<D, KK>;
  const int64_t e = wave * 16 + c;
  const int64_t ee = e < mesh.E ? e : 0;
  const int64_t off = mesh.F * C::NF;
  const double* xf = x + (int64_t)(ix.fid >= 0 ? ix.fid : 0) * C::NF;
  const double* xi = x + off + ee * C::NINT;
#pragma unroll
  for (int kk = 0; kk < C::NK; ++kk) {
    if constexpr (C::NF % 2 == 0 && D == 3) {
      // a lane's facet rows are contiguous: 16-byte loads of row pairs
      if (kk < C::NF) {
        if (kk % 2 == 0) {
          const double2 w = *reinterpret_cast<const double2*>(xf + kk);
          md.x[kk] = w.x;
          md.x[kk + 1] = w.y;
        }
        continue;
      }
    }
    const int t = mass_int_row<D, KK>(kk, g);
    if constexpr (C::NINT > 0) {
      const double* a = mass_is_facet<D, KK>(kk, g) ? xf + kk : xi + (t < C::NINT ? t : C::NINT - 1);
      md.x[kk] = *a;
    } else {
      md.x[kk] = xf[kk < C::NF ? kk : 0];
    }
  }
  const double* Gr = mesh.geo + ee * GEO_STRIDE;
  load_J<D>(Gr, md.J);
  md.det = Gr[GEO_DET];
  md.si = Gr[GEO_SI];
  md.nf = Gr[GEO_NFN + (g <= D ? g : 0)];
  md.ix = ix;
}

// The store of step s: one store instruction per step and lane (a 16-byte
// row pair at even facet steps in 3D with an even facet size, nothing at the
// odd ones); a lane with nothing to write stores to `trash`.  With a fixed
// store count per batch the compiler can wait for the prefetched loads
// without also waiting for these stores.
template <int D, int KK>
constexpr bool mass_pairs() {
  return D == 3 && Cfg<D, KK>::NF % 2 == 0;
}
template <int D, int KK>
__device__ __forceinline__ void mass_store(int s, int g, double v0, double v1, double sfac, double sint, bool fok,
                                           double* fsrow, bool valid, double* irow, double* trash) {
  using C = Cfg<D, KK>;
  if constexpr (mass_pairs<D, KK>()) {
    if (s < C::NF) {
      if (s % 2 == 0)
        *reinterpret_cast<double2*>(fok ? fsrow + s : trash) = make_double2(v0 * sfac, v1 * sfac);
    } else {
      const int t = mass_int_row<D, KK>(s, g);
      *(valid && t < C::NINT ? irow + t : trash) = v0 * sint;
    }
  } else {
    const bool isf = mass_is_facet<D, KK>(s, g);
    const int t = mass_int_row<D, KK>(s, g);
    const bool ok = isf ? fok : valid && t < C::NINT;
    *(ok ? (isf ? fsrow + s : irow + t) : trash) = v0 * (isf ? sfac : sint);
  }
}
// at least as many store instructions as one batch issues (NK), to distinct
// trash slots (so that none is dropped as overwritten)
template <int NK>
__device__ __forceinline__ void mass_dummy_stores(double* trash) {
#pragma unroll
  for (int s = 0; s < NK; ++s) trash[2 + 2 * s] = 0.0;
}
constexpr int64_t MASS_TRASH_DOUBLES = 128;  // >= 2 + 2 NK for every order

// One batch from registers and the fragment tables; writes the outputs and
// returns this lane's share of x_T . y_T.
// T: the MFMA precision of the two contractions (the FP32 form is used for
// the preconditioner of the mixed-precision substeps; everything around the
// contractions stays FP64).
template <typename T, int D, int KK, int MODE>
__device__ __forceinline__ double mass_compute(const MassData<D, KK>& md,
                                               double* __restrict__ out, double* __restrict__ fs,
                                               double* __restrict__ trash, const DevMesh& mesh,
                                               const T* __restrict__ fi, const T* __restrict__ fo,
                                               int64_t wave, int lane, bool live = true) {
  using C = Cfg<D, KK>;
  using M = MF<T>;
  using V = typename M::V;
  const int g = lane >> 4, c = lane & 15;
  const int64_t off = mesh.F * C::NF;
  const int64_t e = wave * 16 + c;
  const bool valid = live && e < mesh.E;  // (a batch that is not live writes nothing)
  // facet rows scaled by |N_F| (mode 1: 1/2 |N_F|^-1, the facet split
  // included), interior rows by the interior scale (its inverse)
  const double sfac = MODE == 1 ? 0.5 / md.nf : md.nf;
  const double sint = MODE == 1 ? 1.0 / md.si : md.si;
  // the lane's facet exists (an interior facet of a real element)
  const bool fok = valid && g <= D && md.ix.fid >= 0;
  T xh[C::NK];
#pragma unroll
  for (int kk = 0; kk < C::NK; ++kk) {
    const bool ok = mass_is_facet<D, KK>(kk, g) ? fok : valid && mass_int_row<D, KK>(kk, g) < C::NINT;
    xh[kk] = (T)(ok ? md.x[kk] * (mass_is_facet<D, KK>(kk, g) ? sfac : sint) : 0.0);
  }
  // Both contractions run their output tiles side by side (independent
  // accumulators) and read the table fragments of the next step while the
  // MFMAs of the current one run.
  double y[C::NMT][4];
  {
    V acc[C::NMT];
    T a[MASS_PF + 1][C::NMT];
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt) acc[mt] = vzero<V>();
#pragma unroll
    for (int kk = 0; kk < MASS_PF && kk < C::NK; ++kk)
#pragma unroll
      for (int mt = 0; mt < C::NMT; ++mt) a[kk][mt] = fi[(mt * C::NK + kk) * 64 + lane];
#pragma unroll
    for (int kk = 0; kk < C::NK; ++kk) {
      if (kk + MASS_PF < C::NK) {
#pragma unroll
        for (int mt = 0; mt < C::NMT; ++mt)
          a[(kk + MASS_PF) % (MASS_PF + 1)][mt] = fi[(mt * C::NK + kk + MASS_PF) * 64 + lane];
      }
      MASS_SCHED_FENCE();
#pragma unroll
      for (int mt = 0; mt < C::NMT; ++mt) acc[mt] = M::mma(a[kk % (MASS_PF + 1)][mt], xh[kk], acc[mt]);
      MASS_SCHED_FENCE();
    }
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) y[mt][i] = (double)acc[mt][i];
  }
  if constexpr (MODE >= 2) {
    // the modal coefficients m = Dinv S x themselves (rho layout; register
    // i of lane group g holds row 16 mt + 4 i + g), stored as double (2) or
    // float (3); a fixed number of stores, the unused ones to trash slots
#pragma unroll
    for (int mt = 0; mt < C::NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * mt + M::row(i, g);
        const bool ok = valid && row < C::NM;
        double* const t = trash + 2 + 2 * (4 * mt + i);
        if constexpr (MODE == 2)
          *(ok ? out + (valid ? e : 0) * C::NM + row : t) = y[mt][i];
        else
          *(ok ? reinterpret_cast<float*>(out) + (valid ? e : 0) * C::NM + row : reinterpret_cast<float*>(t)) =
              (float)y[mt][i];
      }
    return 0.0;
  }
  // component mixing: quads rq = blk*D + a hold components a of one alpha block
  double Gm[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int bb = 0; bb < D; ++bb) {
      double s = 0;
#pragma unroll
      for (int r2 = 0; r2 < D; ++r2) s += md.J[r2][a] * md.J[r2][bb];
      Gm[a][bb] = s;
    }
  double Gs[D][D];
  const double sd = 1.0 / fabs(md.det);
  if (MODE == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) Gs[a][bb] = Gm[a][bb] * sd;
  } else {
    // G^-1 |det| = adj(G)/det(G) |det| = adj(G)/|det|  (det G = det^2)
    if (D == 2) {
      Gs[0][0] = Gm[1][1] * sd; Gs[1][1] = Gm[0][0] * sd;
      Gs[0][1] = -Gm[0][1] * sd; Gs[1][0] = -Gm[1][0] * sd;
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int bb = 0; bb < D; ++bb) {
          const int a1 = (bb + 1) % 3, a2 = (bb + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
          Gs[a][bb] = (Gm[a1][b1] * Gm[a2][b2] - Gm[a1][b2] * Gm[a2][b1]) * sd;
        }
    }
  }
  // in place: quads blk*D .. blk*D + D-1 only mix among themselves.  With
  // m the modal rows before and t after the mix, x_T . y_T = m . t (the two
  // outer factors of the sandwich are transposes of each other), which is
  // this lane's share of the inner product.
  double dot = 0.0;
#pragma unroll
  for (int blk = 0; blk < C::NPK; ++blk) {
    double t[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double s = 0;
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        const int rq = blk * D + bb;
        s += Gs[a][bb] * y[rq / 4][rq % 4];
      }
      t[a] = s;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dot += y[(blk * D + a) / 4][(blk * D + a) % 4] * t[a];
      y[(blk * D + a) / 4][(blk * D + a) % 4] = t[a];
    }
  }
  double* const fsrow = fs + ((int64_t)md.ix.side * mesh.F + (md.ix.fid >= 0 ? md.ix.fid : 0)) * C::NF;
  double* const irow = out + off + (valid ? e : 0) * C::NINT;
  V o[C::NJT];
  {
    T b[MASS_PF + 1][C::NJT];
#pragma unroll
    for (int jt = 0; jt < C::NJT; ++jt) o[jt] = vzero<V>();
#pragma unroll
    for (int rq = 0; rq < MASS_PF && rq < C::NMQ; ++rq)
#pragma unroll
      for (int jt = 0; jt < C::NJT; ++jt) b[rq][jt] = fo[(jt * C::NMQ + rq) * 64 + lane];
#pragma unroll
    for (int rq = 0; rq < C::NMQ; ++rq) {
      if (rq + MASS_PF < C::NMQ) {
#pragma unroll
        for (int jt = 0; jt < C::NJT; ++jt)
          b[(rq + MASS_PF) % (MASS_PF + 1)][jt] = fo[(jt * C::NMQ + rq + MASS_PF) * 64 + lane];
      }
      MASS_SCHED_FENCE();
#pragma unroll
      for (int jt = 0; jt < C::NJT; ++jt) o[jt] = M::mma(b[rq % (MASS_PF + 1)][jt], (T)y[rq / 4][rq % 4], o[jt]);
      MASS_SCHED_FENCE();
    }
  }
#pragma unroll
  for (int jt = 0; jt < C::NJT; ++jt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // output register i of tile jt holds step s = 4 jt + i of this lane
      const int s = 4 * jt + i;
      if (s < C::NK) {
        mass_store<D, KK>(s, g, (double)o[jt][i], i % 2 == 0 && i < 3 ? (double)o[jt][i + 1] : 0.0, sfac, sint, fok,
                          fsrow, valid, irow, trash);
      }
    }
  }
  return dot;
}

// block sum of one double per lane (256 lanes), fixed order; lane 0 of the
// block gets the total
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double red[4];
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// the same over the NW waves of a block (64 NW lanes): per-wave sums, then
// pairwise in a fixed order
template <int NW>
__device__ __forceinline__ double block_sum_waves(double v) {
  __shared__ double red[NW];
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) t[i] = red[i];
#pragma unroll
  for (int w = 1; w < NW; w *= 2)
#pragma unroll
    for (int i = 0; i < NW; i += 2 * w) t[i] = t[i] + t[i + w];
  return t[0];
}

// one batch per wave
// part (nullable): per-block partial of x . y
template <int D, int KK, int MODE>
__global__ __launch_bounds__(256) void k_mass(const double* __restrict__ x, double* __restrict__ out,
                                              double* __restrict__ fs, DevMesh mesh,
                                              const double* __restrict__ fin,
                                              const double* __restrict__ fout,
                                              const int* __restrict__ flag, double* __restrict__ part) {
  if (flag && *flag) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double dot = 0.0;
  if (wave * 16 < mesh.E) {
    MassIdx ix;
    MassData<D, KK> md;
    mass_load_idx<D>(mesh, wave, lane >> 4, lane & 15, ix);
    mass_load_data<D, KK>(x, mesh, wave, lane >> 4, lane & 15, ix, md);
    dot = mass_compute<double, D, KK, MODE>(md, out, fs, fs + 2 * mesh.F * Cfg<D, KK>::NF, mesh, fin, fout, wave,
                                            lane);
  }
  if (part) {
    dot = block_sum256(dot);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
  }
}

// Persistent variant for orders whose two tables fit in LDS: each block
// copies the tables to LDS once, then its waves walk batches with a grid
// stride and gather the next batch while the current batch's MFMAs run
// (table fragments come from LDS, so the in-order vector-memory counter only
// tracks the gathers).
template <int D, int KK>
constexpr int mass_lds_doubles() {
  using C = Cfg<D, KK>;
  return (C::NMT * C::NK + C::NJT * C::NMQ) * 64;
}

template <typename T, int D, int KK, int MODE>
__global__ __launch_bounds__(64 * MASS_WPB, 1) void k_mass_lds(const double* __restrict__ x, double* __restrict__ out,
                                                  double* __restrict__ fs, DevMesh mesh,
                                                  const T* __restrict__ fin,
                                                  const T* __restrict__ fout,
                                                  const int* __restrict__ flag, double* __restrict__ part) {
  using C = Cfg<D, KK>;
  extern __shared__ double lds_raw[];
  T* const lds = reinterpret_cast<T*>(lds_raw);
  if (flag && *flag) return;  // uniform over the launch
  constexpr int NIN = C::NMT * C::NK * 64;
  // table entries (of type T); the modal modes use the first table only
  constexpr int NTOT = MODE >= 2 ? NIN : mass_lds_doubles<D, KK>();
  for (int i = threadIdx.x; i < NTOT; i += 64 * MASS_WPB) lds[i] = i < NIN ? fin[i] : fout[i - NIN];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  // Each XCD (blocks are dealt round-robin over the 8) walks a contiguous
  // range of batches, so that elements sharing a facet, mostly close in
  // numbering, read its rows through the same L2.
  const int nx = gridDim.x % 8 == 0 ? 8 : 1;
  const int64_t xcd = blockIdx.x % nx;
  const int64_t nw_all = (mesh.E + 15) / 16;
  const int64_t nw = nw_all * (xcd + 1) / nx;  // end of this XCD's range
  const int64_t stride = (int64_t)(gridDim.x / nx) * MASS_WPB;
  int64_t wave = nw_all * xcd / nx + (int64_t)(blockIdx.x / nx) * MASS_WPB + (threadIdx.x >> 6);
  double dot = 0.0;
  // Two register sets alternate (no copy between them).  Every load and
  // store is issued unconditionally (prefetches past the last batch read
  // clamped, in-range addresses; a batch past the end computes zeros and
  // stores them to the trash slot), and the prologue issues the stores of
  // one batch to the trash slot, so the loop is entered with the same
  // vector-memory history as it repeats with: the wait at the top (for the
  // facet ids that address the next gather) then lets the previous batch's
  // stores stay in flight.  There is no exit between a prefetch and its use,
  // which would let the compiler sink the prefetch to the use.
  double* const trash = fs + 2 * mesh.F * C::NF;
  MassIdx ib;
  MassData<D, KK> da, db;
  if (wave < nw) {
    mass_load_idx<D>(mesh, wave, g, c, ib);
    mass_load_data<D, KK>(x, mesh, wave, g, c, ib, da);
    mass_load_idx<D>(mesh, wave + stride, g, c, ib);
    asm volatile("" ::: "memory");  // the dummy stores follow the loads
    mass_dummy_stores<(MODE >= 2 ? 4 * C::NMT : C::NK)>(trash);
    while (true) {
      mass_load_data<D, KK>(x, mesh, wave + stride, g, c, ib, db);
      mass_load_idx<D>(mesh, wave + 2 * stride, g, c, ib);
      // opaque base: keeps the fragment reads inside the loop instead of
      // hoisting all of them into registers
      int base = 0;
      asm volatile("" : "+s"(base));
      dot += mass_compute<T, D, KK, MODE>(da, out, fs, trash, mesh, lds + base, lds + base + NIN, wave, lane);
      mass_load_data<D, KK>(x, mesh, wave + 2 * stride, g, c, ib, da);
      mass_load_idx<D>(mesh, wave + 3 * stride, g, c, ib);
      asm volatile("" : "+s"(base));
      dot += mass_compute<T, D, KK, MODE>(db, out, fs, trash, mesh, lds + base, lds + base + NIN, wave + stride,
                                          lane, wave + stride < nw);
      wave += 2 * stride;
      if (wave >= nw) break;
    }
  }
  if (part) {
    dot = block_sum_waves<MASS_WPB>(dot);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
  }
}

// Streamed-table variant for orders whose two tables do not fit in LDS
// (3D k = 4: 197 KB, k = 5: 484 KB in FP64).  A block of TILE_WPB waves
// walks TILE_WPB batches per round in lock step; the tables pass through a
// double-buffered LDS window in chunks, each chunk copied once per block
// (from L2) and read by all its waves, so the table traffic per batch drops
// TILE_WPB-fold against one read per wave.  While the MFMAs of one chunk
// run, every thread holds its share of the next chunk in registers and
// stores it to the other buffer after them; one barrier per chunk.  Each
// contraction runs in two passes over halves of its output tiles (the
// accumulators of all tiles and the operand rows would not fit in the 256
// registers of a kernel with two waves per SIMD); a chunk holds K steps of
// one half, so every table entry is still copied once per round.
// Every wave of a block runs the same number of rounds and chunks (a batch
// past the end computes on clamped addresses and writes nothing).  A
// round's gather (a few microseconds) against its ~50 microseconds of MFMA
// work is left exposed: there are no registers for a prefetch.
static constexpr int TILE_WPB = 8;

template <int D, int KK>
struct MassTile {
  using C = Cfg<D, KK>;
  // halves of the output tiles of each contraction
  static constexpr int H1 = (C::NMT + 1) / 2;  // tiles of the first pass
  static constexpr int H2 = (C::NJT + 1) / 2;
  // steps per chunk, and chunks per pass
  static constexpr int K1 = 7;
  static constexpr int K2 = 8;
  static constexpr int N1 = (C::NK + K1 - 1) / K1;
  static constexpr int N2 = (C::NMQ + K2 - 1) / K2;
  static constexpr int NCH = 2 * N1 + 2 * N2;  // chunks per round
  static constexpr int CH1 = K1 * H1 * 64;     // doubles per chunk (largest of each kind)
  static constexpr int CH2 = K2 * H2 * 64;
  static constexpr int CH = CH1 > CH2 ? CH1 : CH2;
  static constexpr int PER = (CH + 64 * TILE_WPB - 1) / (64 * TILE_WPB);  // per thread
};

// Chunk c of a round (c mod NCH): the first contraction's passes p = 0, 1
// (chunks p N1 + j, steps j K1 ..), then the second's (2 N1 + p N2 + j).
// Laid out [step - first step][tile - first tile][lane].
template <typename T, int D, int KK>
struct TileChunk {
  const T* src;
  int nk, k0, nks, t0, nts;  // table K size; first step and steps; first tile and tiles
  __device__ __forceinline__ TileChunk(const T* fin, const T* fout, int c) {
    using C = Cfg<D, KK>;
    using TT = MassTile<D, KK>;
    c %= TT::NCH;
    const bool first = c < 2 * TT::N1;
    const int cc = first ? c : c - 2 * TT::N1;
    const int n = first ? TT::N1 : TT::N2, kc = first ? TT::K1 : TT::K2;
    const int p = cc / n, j = cc - p * n;
    const int half = first ? TT::H1 : TT::H2, nt = first ? C::NMT : C::NJT;
    src = first ? fin : fout;
    nk = first ? C::NK : C::NMQ;
    k0 = j * kc;
    nks = nk - k0 < kc ? nk - k0 : kc;
    t0 = p * half;
    nts = nt - t0 < half ? nt - t0 : half;
  }
};

template <typename T, int D, int KK>
__device__ __forceinline__ void tile_fetch(const T* __restrict__ fin, const T* __restrict__ fout, int c,
                                           T (&st)[MassTile<D, KK>::PER]) {
  using TT = MassTile<D, KK>;
  const TileChunk<T, D, KK> k(fin, fout, c);
  // an opaque copy of the base: the chunk's addresses do not depend on the
  // round, and the compiler would otherwise hoist every round's loads out of
  // the loop and hold all chunks in registers
  const T* src = k.src;
  asm volatile("" : "+s"(src));
  int tid = (int)threadIdx.x;  // (likewise the per-thread offsets)
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int p = 0; p < TT::PER; ++p) {
    const int i = tid + p * 64 * TILE_WPB;
    const int s = i / (k.nts * 64), rem = i - s * k.nts * 64;
    const int t = k.t0 + (rem >> 6), l = rem & 63;
    const bool ok = s < k.nks;
    st[p] = src[ok ? (((t * k.nk + k.k0 + s) << 6) + l) : 0];
  }
}
template <typename T, int D, int KK>
__device__ __forceinline__ void tile_store(T* __restrict__ buf, const T (&st)[MassTile<D, KK>::PER]) {
#pragma unroll
  for (int p = 0; p < MassTile<D, KK>::PER; ++p) {
    const int i = (int)threadIdx.x + p * 64 * TILE_WPB;
    if (i < MassTile<D, KK>::CH) buf[i] = st[p];
  }
}

// One pass of a contraction over tiles [T0, T0 + NT) of its output, K steps
// 0 .. NKT in chunks of KC from the LDS window: acc[t] += A(step, T0 + t) b[step].
// c: the round's index of the pass's first chunk; cb: the buffer holding it.
template <typename T, int D, int KK, int NT, int NKT, int KC, int NB>
__device__ __forceinline__ void tile_pass(const T* __restrict__ fin, const T* __restrict__ fout,
                                          T (*buf)[MassTile<D, KK>::CH], int c, int& cb,
                                          T (&st)[MassTile<D, KK>::PER], const T (&b)[NB],
                                          typename MF<T>::V (&acc)[NT], int lane) {
  using M = MF<T>;
  constexpr int NCHK = (NKT + KC - 1) / KC;
#pragma unroll
  for (int ch = 0; ch < NCHK; ++ch) {
    tile_fetch<T, D, KK>(fin, fout, c + ch + 1, st);  // the round's next chunk
    const T* const a = buf[cb];
    const int nks = NKT - ch * KC < KC ? NKT - ch * KC : KC;
    T fr[2][NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) fr[0][t] = a[t * 64 + lane];
#pragma unroll
    for (int s = 0; s < KC; ++s) {
      if (s < nks) {
        if (s + 1 < nks) {
#pragma unroll
          for (int t = 0; t < NT; ++t) fr[(s + 1) & 1][t] = a[((s + 1) * NT + t) * 64 + lane];
        }
        MASS_SCHED_FENCE();
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = M::mma(fr[s & 1][t], b[ch * KC + s], acc[t]);
        MASS_SCHED_FENCE();
      }
    }
    tile_store<T, D, KK>(buf[cb ^ 1], st);
    cb ^= 1;
    __syncthreads();
  }
}

// T: the MFMA precision of the two contractions (FP32 for the preconditioner
// of the mixed-precision substeps, with the FP32 row-map tables; the
// gather, the mixing and the stores stay FP64).
template <typename T, int D, int KK, int MODE>
__global__ __launch_bounds__(64 * TILE_WPB, 1) void k_mass_tiled(const double* __restrict__ x,
                                                                 double* __restrict__ out, double* __restrict__ fs,
                                                                 DevMesh mesh, const T* __restrict__ fin,
                                                                 const T* __restrict__ fout,
                                                                 const int* __restrict__ flag,
                                                                 double* __restrict__ part) {
  using C = Cfg<D, KK>;
  using TT = MassTile<D, KK>;
  using VT = typename MF<T>::V;
  static_assert(D == 3, "the streamed-table kernel serves the 3D orders only");
  __shared__ T buf[2][TT::CH];
  if (flag && *flag) return;  // uniform over the launch
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int nx = gridDim.x % 8 == 0 ? 8 : 1;
  const int64_t xcd = blockIdx.x % nx;
  const int64_t nw_all = (mesh.E + 15) / 16;
  const int64_t lo = nw_all * xcd / nx, hi = nw_all * (xcd + 1) / nx;
  const int64_t per_round = (int64_t)(gridDim.x / nx) * TILE_WPB;
  const int64_t rounds = (hi - lo + per_round - 1) / per_round;
  const int64_t first = lo + (int64_t)(blockIdx.x / nx) * TILE_WPB + (threadIdx.x >> 6);
  const int64_t off = mesh.F * C::NF;
  double* const trash = fs + 2 * mesh.F * C::NF;
  double dot = 0.0;
  T st[TT::PER];
  tile_fetch<T, D, KK>(fin, fout, 0, st);  // the round's first chunk
  tile_store<T, D, KK>(buf[0], st);
  __syncthreads();
  int cb = 0;  // the buffer holding the chunk about to be used
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t wave = first + r * per_round;
    const bool live = wave < hi;
    MassIdx ix;
    MassData<D, KK> md;
    mass_load_idx<D>(mesh, live ? wave : lo, g, c, ix);
    mass_load_data<D, KK>(x, mesh, live ? wave : lo, g, c, ix, md);
    const int64_t e = wave * 16 + c;
    const bool valid = live && e < mesh.E;
    const double sfac = MODE == 1 ? 0.5 / md.nf : md.nf;
    const double sint = MODE == 1 ? 1.0 / md.si : md.si;
    const bool fok = valid && g <= D && md.ix.fid >= 0;
    T xh[C::NK];
#pragma unroll
    for (int kk = 0; kk < C::NK; ++kk) {
      const bool ok = mass_is_facet<D, KK>(kk, g) ? fok : valid && mass_int_row<D, KK>(kk, g) < C::NINT;
      xh[kk] = (T)(ok ? md.x[kk] * (mass_is_facet<D, KK>(kk, g) ? sfac : sint) : 0.0);
    }
    // ---- first contraction y = fin . xh, in two passes over its tiles
    double y[C::NMT][4];
    {
      VT acc[TT::H1];
#pragma unroll
      for (int t = 0; t < TT::H1; ++t) acc[t] = vzero<VT>();
      tile_pass<T, D, KK, TT::H1, C::NK, TT::K1, C::NK>(fin, fout, buf, 0, cb, st, xh, acc, lane);
#pragma unroll
      for (int t = 0; t < TT::H1; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[t][i] = (double)acc[t][i];
    }
    {
      constexpr int NT = C::NMT - TT::H1;
      VT acc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = vzero<VT>();
      tile_pass<T, D, KK, NT, C::NK, TT::K1, C::NK>(fin, fout, buf, TT::N1, cb, st, xh, acc, lane);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[TT::H1 + t][i] = (double)acc[t][i];
    }
    // ---- component mixing (as in mass_compute) and the local x . y share;
    // the geometry is read again here rather than held through the MFMAs
    {
      const double* Gr = mesh.geo + (live ? wave * 16 + c < mesh.E ? wave * 16 + c : 0 : lo * 16) * GEO_STRIDE;
      load_J<D>(Gr, md.J);
      md.det = Gr[GEO_DET];
    }
    double Gm[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        double s = 0;
#pragma unroll
        for (int r2 = 0; r2 < D; ++r2) s += md.J[r2][a] * md.J[r2][bb];
        Gm[a][bb] = s;
      }
    double Gs[D][D];
    const double sd = 1.0 / fabs(md.det);
    if (MODE == 0) {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int bb = 0; bb < D; ++bb) Gs[a][bb] = Gm[a][bb] * sd;
    } else {
      // G^-1 |det| = adj(G) / |det|  (det G = det^2)
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int bb = 0; bb < D; ++bb) {
          const int a1 = (bb + 1) % 3, a2 = (bb + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
          Gs[a][bb] = (Gm[a1][b1] * Gm[a2][b2] - Gm[a1][b2] * Gm[a2][b1]) * sd;
        }
    }
    T yb[C::NMQ];  // the mixed rows, by step of the second contraction
#pragma unroll
    for (int blk = 0; blk < C::NPK; ++blk) {
      double t[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s = 0;
#pragma unroll
        for (int bb = 0; bb < D; ++bb) {
          const int rq = blk * D + bb;
          s += Gs[a][bb] * y[rq / 4][rq % 4];
        }
        t[a] = s;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        dot += y[(blk * D + a) / 4][(blk * D + a) % 4] * t[a];
        yb[blk * D + a] = (T)t[a];
      }
    }
#pragma unroll
    for (int rq = D * C::NPK; rq < C::NMQ; ++rq) yb[rq] = (T)0;
    // ---- second contraction o = fout . yb, in two passes, stored per pass
    double* const fsrow = fs + ((int64_t)md.ix.side * mesh.F + (md.ix.fid >= 0 ? md.ix.fid : 0)) * C::NF;
    double* const irow = out + off + (valid ? e : 0) * C::NINT;
    auto store = [&](const VT& ot, int jt) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int s = 4 * jt + i;  // register i of tile jt holds step s of this lane
        if (s < C::NK)
          mass_store<D, KK>(s, g, (double)ot[i], i % 2 == 0 && i < 3 ? (double)ot[i + 1] : 0.0, sfac, sint, fok,
                            fsrow, valid, irow, trash);
      }
    };
    {
      VT o[TT::H2];
#pragma unroll
      for (int t = 0; t < TT::H2; ++t) o[t] = vzero<VT>();
      tile_pass<T, D, KK, TT::H2, C::NMQ, TT::K2, C::NMQ>(fin, fout, buf, 2 * TT::N1, cb, st, yb, o, lane);
#pragma unroll
      for (int t = 0; t < TT::H2; ++t) store(o[t], t);
    }
    {
      constexpr int NT = C::NJT - TT::H2;
      VT o[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) o[t] = vzero<VT>();
      tile_pass<T, D, KK, NT, C::NMQ, TT::K2, C::NMQ>(fin, fout, buf, 2 * TT::N1 + TT::N2, cb, st, yb, o, lane);
#pragma unroll
      for (int t = 0; t < NT; ++t) store(o[t], TT::H2 + t);
    }
  }
  if (part) {
    dot = block_sum_waves<TILE_WPB>(dot);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
  }
}

// facet rows: r_F = slot(T) + slot(T'), lower element first (deterministic)
template <int NF, int NFL>
__global__ void k_assemble_flag(double* __restrict__ r, const double* __restrict__ slot, DevMesh mesh,
                                const int* __restrict__ flag) {
  if (flag && *flag) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mesh.F * NF) return;
  const int64_t F = t / NF;
  const int jj = (int)(t - F * NF);
  const int32_t e0 = mesh.facet_elem[2 * F], e1 = mesh.facet_elem[2 * F + 1];
  const int i0 = mesh.facet_local[2 * F], i1 = mesh.facet_local[2 * F + 1];
  r[t] = slot[(int64_t)e0 * NFL + i0 * NF + jj] + slot[(int64_t)e1 * NFL + i1 * NF + jj];
}

// facet rows from the facet-side buffer: v_F = fs[0][F] + fs[1][F]
__global__ void k_fs_assemble(double* __restrict__ v, const double* __restrict__ fs, int64_t nfl,
                              const int* __restrict__ flag) {
  if (flag && *flag) return;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nfl; t += (int64_t)gridDim.x * 256)
    v[t] = fs[t] + fs[nfl + t];
}

// ------------------------------------------------------------------ launchers
void launch_fs_assemble(hipStream_t s, double* v, const double* fs, int64_t nfl, const int* flag) {
  if (nfl <= 0) return;
  const int64_t b = std::min<int64_t>((nfl + 255) / 256, 2048);
  hipLaunchKernelGGL(k_fs_assemble, dim3((unsigned)b), dim3(256), 0, s, v, fs, nfl, flag);
}

template <typename T, int D, int KK>
void launch_modal(hipStream_t s, const double* x, T* m, const DevMesh& mesh, const double* frag) {
  const int64_t waves = (mesh.E + 15) / 16;
  const int64_t blocks = (waves + 3) / 4;
  HOPU_LAUNCH((k_modal<T, D, KK>), dim3((unsigned)blocks), dim3(256), 0, s, x, m, mesh, frag);
}

template <typename T, int D, int KK>
void launch_elem(hipStream_t s, const T* m, double* r, double* slot, const DevMesh& mesh,
                 const DevTables<T>& tb, int terms, double* diss_part, double* eta_nd) {
  HOPU_LAUNCH((k_elem<T, D, KK>), dim3((unsigned)mesh.nb), dim3(64), 0, s, m, r, slot, mesh, tb, terms, diss_part,
              eta_nd);
}
template <int NS, int D, int KK>
void launch_elem_bf(hipStream_t s, const float* m, double* r, double* slot, const DevMesh& mesh,
                    const DevTables<BfPack<NS>>& tb, int terms, double* diss_part) {
  HOPU_LAUNCH((k_elem<float, D, KK, NS>), dim3((unsigned)mesh.nb), dim3(64), 0, s, m, r, slot, mesh, tb, terms,
              diss_part, nullptr);
}

template <int D, int KK>
void launch_assemble(hipStream_t s, double* r, const double* slot, const DevMesh& mesh, const int* flag) {
  using C = Cfg<D, KK>;
  const int64_t n = mesh.F * C::NF;
  if (n > 0)
    hipLaunchKernelGGL((k_assemble_flag<C::NF, C::NFL>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r,
                       slot, mesh, flag);
}

template <int D, int KK>
int launch_mass(hipStream_t s, int mode, const double* x, double* out, double* fs, const DevMesh& mesh,
                const double* fin, const double* fout, const int* flag, double* part, const float* fin32,
                const float* fout32) {
  using C = Cfg<D, KK>;
  const int64_t waves = (mesh.E + 15) / 16;
  constexpr size_t lds_bytes = (size_t)mass_lds_doubles<D, KK>() * sizeof(double);
  if (waves == 0) return 0;
  if constexpr (lds_bytes <= 64 * 1024) {
    // one block of MASS_WPB waves per CU (the tables take up to 64 KB of LDS)
    const int64_t blocks = std::min<int64_t>((waves + MASS_WPB - 1) / MASS_WPB, MASS_BLOCKS);
    const dim3 thr(64 * MASS_WPB);
    if (mode == 0)
      HOPU_LAUNCH((k_mass_lds<double, D, KK, 0>), dim3((unsigned)blocks), thr, lds_bytes, s, x, out, fs, mesh, fin,
                  fout, flag, part);
    else if (fin32 && fout32)
      HOPU_LAUNCH((k_mass_lds<float, D, KK, 1>), dim3((unsigned)blocks), thr, lds_bytes / 2, s, x, out, fs, mesh,
                  fin32, fout32, flag, part);
    else
      HOPU_LAUNCH((k_mass_lds<double, D, KK, 1>), dim3((unsigned)blocks), thr, lds_bytes, s, x, out, fs, mesh, fin,
                  fout, flag, part);
    return (int)blocks;
  } else if constexpr (D == 3) {
    // tables streamed through LDS by blocks of TILE_WPB waves (one block
    // per CU)
    const int64_t blocks = std::min<int64_t>((waves + TILE_WPB - 1) / TILE_WPB, MASS_BLOCKS);
    const dim3 thr(64 * TILE_WPB);
    if (mode == 0)
      HOPU_LAUNCH((k_mass_tiled<double, D, KK, 0>), dim3((unsigned)blocks), thr, 0, s, x, out, fs, mesh, fin, fout,
                  flag, part);
    else if (fin32 && fout32)
      HOPU_LAUNCH((k_mass_tiled<float, D, KK, 1>), dim3((unsigned)blocks), thr, 0, s, x, out, fs, mesh, fin32,
                  fout32, flag, part);
    else
      HOPU_LAUNCH((k_mass_tiled<double, D, KK, 1>), dim3((unsigned)blocks), thr, 0, s, x, out, fs, mesh, fin, fout,
                  flag, part);
    (void)sizeof(C);
    return (int)blocks;
  } else {
    const int64_t blocks = (waves + 3) / 4;
    if (mode == 0)
      HOPU_LAUNCH((k_mass<D, KK, 0>), dim3((unsigned)blocks), dim3(256), 0, s, x, out, fs, mesh, fin, fout, flag,
                  part);
    else
      HOPU_LAUNCH((k_mass<D, KK, 1>), dim3((unsigned)blocks), dim3(256), 0, s, x, out, fs, mesh, fin, fout, flag,
                  part);
    (void)sizeof(C);
    (void)fin32;
    (void)fout32;
    return (int)blocks;
  }
}

// m = Dinv S x through the persistent mass kernel (its gather, row order
// and first contraction; modes 2/3 store m as double/float).  false: this
// order's table does not fit in LDS (the caller uses k_modal).
template <int D, int KK>
bool launch_modal_mass(hipStream_t s, const double* x, void* m, bool f32, double* fs, const DevMesh& mesh,
                       const double* fin) {
  using C = Cfg<D, KK>;
  constexpr size_t lds_bytes = (size_t)C::NMT * C::NK * 64 * sizeof(double);
  if constexpr (lds_bytes <= 64 * 1024 && 2 + 8 * C::NMT <= MASS_TRASH_DOUBLES) {
    const int64_t waves = (mesh.E + 15) / 16;
    if (waves == 0) return true;
    const int64_t blocks = std::min<int64_t>((waves + MASS_WPB - 1) / MASS_WPB, MASS_BLOCKS);
    const dim3 thr(64 * MASS_WPB);
    double* out = static_cast<double*>(m);
    if (f32)
      HOPU_LAUNCH((k_mass_lds<double, D, KK, 3>), dim3((unsigned)blocks), thr, lds_bytes, s, x, out, fs, mesh, fin,
                  fin, nullptr, nullptr);
    else
      HOPU_LAUNCH((k_mass_lds<double, D, KK, 2>), dim3((unsigned)blocks), thr, lds_bytes, s, x, out, fs, mesh, fin,
                  fin, nullptr, nullptr);
    return true;
  } else {
    (void)s; (void)x; (void)m; (void)f32; (void)fs; (void)mesh; (void)fin;
    return false;
  }
}

#define HOPU_INST(D, KK)                                                                                     \
  template void launch_modal<double, D, KK>(hipStream_t, const double*, double*, const DevMesh&,            \
                                            const double*);                                                 \
  template void launch_modal<float, D, KK>(hipStream_t, const double*, float*, const DevMesh&,              \
                                           const double*);                                                  \
  template void launch_elem<double, D, KK>(hipStream_t, const double*, double*, double*, const DevMesh&,    \
                                           const DevTables<double>&, int, double*, double*);                \
  template void launch_elem<float, D, KK>(hipStream_t, const float*, double*, double*, const DevMesh&,      \
                                          const DevTables<float>&, int, double*, double*);                  \
  template void launch_elem_bf<2, D, KK>(hipStream_t, const float*, double*, double*, const DevMesh&,       \
                                         const DevTables<BfPack<2>>&, int, double*);                        \
  template void launch_elem_bf<3, D, KK>(hipStream_t, const float*, double*, double*, const DevMesh&,       \
                                         const DevTables<BfPack<3>>&, int, double*);                        \
  template int launch_mass<D, KK>(hipStream_t, int, const double*, double*, double*, const DevMesh&,        \
                                  const double*, const double*, const int*, double*, const float*,          \
                                  const float*);                                                            \
  template void launch_assemble<D, KK>(hipStream_t, double*, const double*, const DevMesh&, const int*);        \
  template bool launch_modal_mass<D, KK>(hipStream_t, const double*, void*, bool, double*, const DevMesh&,   \
                                         const double*);

HOPU_INST(2, 1)
HOPU_INST(2, 2)
HOPU_INST(2, 3)
HOPU_INST(2, 4)
HOPU_INST(3, 1)
HOPU_INST(3, 2)
HOPU_INST(3, 3)
HOPU_INST(3, 4)
HOPU_INST(3, 5)

}  // namespace hopu
