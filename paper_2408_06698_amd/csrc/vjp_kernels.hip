// Transpose Jacobian of the convection residual, out = J_r(u)^T mu.
// With mu_h = sum mu_i phi_i, for each basis function phi_j:
//   - int_T phi_j . (grad mu_h + grad mu_h^T) u
//   + int_E (phi_j.n) s + (u.n) <phi_j>.[[mu]] + 1/2|u.n| (I-Pi)[[phi_j]].(I-Pi)[[mu]]
//   s = <u>.[[mu]] + 1/2 sgn(u.n) (I-Pi)[[u]].(I-Pi)[[mu]],  sgn(0) = 0.
// Each element tests with its own trace from its own side (n its outward
// normal, [[.]] = own - neighbour): h = 1/2 s n + 1/2 (u.n)[[mu]] + (I-Pi)a,
// a = 1/2|u.n|(I-Pi)[[mu]]; the neighbour does the same from its side.
// Batches, tables and fragment layouts are those of the forward kernel;
// NS > 0 (T = float) runs the contractions in split BF16 as the forward
// kernel does (see mma_bf), with two more split tables (vol_dV, vol_VT).
// In the reduced forms u.n at the facet points is computed in FP64 from
// the facet DoFs of the FP64 state (u.n_F = sum_j x_Fj psi_j on the facet,
// by one f64 MFMA per group of four DoFs): sgn(u.n) is a discontinuous
// function of the state, and where |u.n| is below the reduced forms'
// rounding the traces' u.n would flip it against the FP64 result, an O(1)
// change of the facet rows there.  The FP64 form takes u.n from its traces,
// as the residual does.
#include <type_traits>

#include "bf16split.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "launch_events.hpp"

namespace hopu {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct VM;
template <> struct VM<double> {
  typedef d4 V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int g) { return 4 * i + g; }
};
template <> struct VM<float> {
  typedef f4 V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int g) { return 4 * g + i; }
};
template <typename V> __device__ __forceinline__ V vz() { V v = {0, 0, 0, 0}; return v; }

template <typename T, int D, int KK, int NS = 0>
__global__ __launch_bounds__(64) void k_vjp(const T* __restrict__ mu_m, const T* __restrict__ mm_m,
                                             double* __restrict__ out, double* __restrict__ oslot, DevMesh mesh,
                                             DevTables<TabT<T, NS>> tb, const double* __restrict__ udual,
                                             const double* __restrict__ psi_n) {
  using C = Cfg<D, KK>;
  using M = VM<T>;
  using V = typename M::V;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t b = blockIdx.x;  // one wave (batch) per block, as in the forward kernel
  if (b >= mesh.nb) return;
  const int32_t e = mesh.belem[b * 16 + c];
  const bool valid = e >= 0;
  const int64_t ee = valid ? e : mesh.belem[b * 16];
  const int sig = mesh.bsig[b];
  const double* Gr = mesh.geo + ee * GEO_STRIDE;
  double J[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int cc = 0; cc < D; ++cc) J[r][cc] = Gr[r * D + cc];
  const double det = Gr[GEO_DET], idet = 1.0 / det;

  T uB[D][C::NPK], mB[D][C::NPK];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int kk = 0; kk < C::NPK; ++kk) {
      uB[a][kk] = mu_m[ee * C::NM + kk * 4 * D + 4 * a + g];
      mB[a][kk] = mm_m[ee * C::NM + kk * 4 * D + 4 * a + g];
    }
  // split-BF16 form: the element's modal coefficients split once, in groups
  // of four steps
  constexpr int NGP = (C::NPK + 3) / 4;
  BfTab<NS> uS[D][NGP], mS[D][NGP];
  if constexpr (NS > 0) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int sg = 0; sg < NGP; ++sg) {
        uS[a][sg] = bf_steps<NS>(uB[a], 4 * sg);
        mS[a][sg] = bf_steps<NS>(mB[a], 4 * sg);
      }
  }
  double acc[D][C::NAT][4];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int at = 0; at < C::NAT; ++at)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[a][at][i] = 0.0;

  // ---------------- volume: - sgn/det^2 int phi^ . (G (grad^mu^) u^ + (grad^mu^)^T G u^)
  {
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
      V u[D], gm[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        u[a] = vz<V>();
#pragma unroll
        for (int bb = 0; bb < D; ++bb) gm[a][bb] = vz<V>();
      }
      if constexpr (NS == 0) {
#pragma unroll
        for (int kk = 0; kk < C::NPK; ++kk) {
          const T av = tb.vol_V[(qt * C::NPK + kk) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) u[a] = M::mma(av, uB[a][kk], u[a]);
#pragma unroll
          for (int bb = 0; bb < D; ++bb) {
            const T ad = tb.vol_dV[((qt * D + bb) * C::NPK + kk) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) gm[a][bb] = M::mma(ad, mB[a][kk], gm[a][bb]);
          }
        }
      } else {
#pragma unroll
        for (int sg = 0; sg < NGP; ++sg) {
          const BfTab<NS> av = tb.vol_V[(qt * NGP + sg) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) u[a] = mma_bf<NS>(av, uS[a][sg], u[a]);
#pragma unroll
          for (int bb = 0; bb < D; ++bb) {
            const BfTab<NS> ad = tb.vol_dV[((qt * D + bb) * NGP + sg) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) gm[a][bb] = mma_bf<NS>(ad, mS[a][sg], gm[a][bb]);
          }
        }
      }
      T v[D][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 16 * qt + M::row(i, g);
        const double wq = q < C::NQV ? tb.wv[q] : 0.0;
        double uh[D], gu[D], t1[D], vv[D];
#pragma unroll
        for (int a = 0; a < D; ++a) uh[a] = (double)u[a][i];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = 0, s2 = 0;
#pragma unroll
          for (int bb = 0; bb < D; ++bb) { s += Gm[a][bb] * uh[bb]; s2 += (double)gm[a][bb][i] * uh[bb]; }
          gu[a] = s;   // G u^
          t1[a] = s2;  // (grad^ mu^) u^
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = 0, s2 = 0;
#pragma unroll
          for (int bb = 0; bb < D; ++bb) { s += Gm[a][bb] * t1[bb]; s2 += (double)gm[bb][a][i] * gu[bb]; }
          vv[a] = (s + s2) * wq * sc;
        }
#pragma unroll
        for (int a = 0; a < D; ++a) v[a][i] = (T)vv[a];
      }
      V t[D][C::NAT];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int at = 0; at < C::NAT; ++at) t[a][at] = vz<V>();
      if constexpr (NS == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int at = 0; at < C::NAT; ++at) {
            const T av = tb.vol_VT[((qt * 4 + i) * C::NAT + at) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) t[a][at] = M::mma(av, v[a][i], t[a][at]);
          }
      } else {
        // the four points i of the tile are one step group
        BfTab<NS> vb[D];
#pragma unroll
        for (int a = 0; a < D; ++a) vb[a] = bf_split4<NS>(v[a][0], v[a][1], v[a][2], v[a][3]);
#pragma unroll
        for (int at = 0; at < C::NAT; ++at) {
          const BfTab<NS> av = tb.vol_VT[(qt * C::NAT + at) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) t[a][at] = mma_bf<NS>(av, vb[a], t[a][at]);
        }
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int at = 0; at < C::NAT; ++at)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[a][at][i] += (double)t[a][at][i];
    }
  }

  // ---------------- facets
#pragma unroll 1
  for (int f = 0; f <= D; ++f) {
    const int fp = (sig >> (4 * f)) & 0xF;
    if (fp == 0xF) continue;
    const int32_t en = valid ? mesh.nbr[ee * (D + 1) + f] : (int32_t)ee;
    const double* Gn = mesh.geo + (int64_t)en * GEO_STRIDE;
    double Jn[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int cc = 0; cc < D; ++cc) Jn[r][cc] = Gn[r * D + cc];
    const double idetn = 1.0 / Gn[GEO_DET];
    const double nfn = Gr[GEO_NFN + f];
    double nrm[D];
#pragma unroll
    for (int a = 0; a < D; ++a) nrm[a] = Gr[GEO_NRM + f * D + a];
    int lf = mesh.lglob;
    if (mesh.lfac) lf = valid ? (int)mesh.lfac[mesh.fid[ee * (D + 1) + f]] : -1;
    // the facet DoFs of u, with the sign of this element's outward normal
    // against the facet's own (sigma = (-1)^f sgn det J): lane group g holds
    // DoF 4 jk + g at step jk
    double xF[C::NFK];
    {
      const int64_t Fid = mesh.fid[ee * (D + 1) + f];
      const double sig = ((f & 1) ? -1.0 : 1.0) * (det > 0 ? 1.0 : -1.0);
#pragma unroll
      for (int jk = 0; jk < C::NFK; ++jk) {
        const int j = 4 * jk + g;
        xF[jk] = j < C::NF ? sig * udual[Fid * C::NF + (j < C::NF ? j : 0)] : 0.0;
      }
    }
    T nuB[D][C::NPK], nmB[D][C::NPK];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int kk = 0; kk < C::NPK; ++kk) {
        nuB[a][kk] = mu_m[(int64_t)en * C::NM + kk * 4 * D + 4 * a + g];
        nmB[a][kk] = mm_m[(int64_t)en * C::NM + kk * 4 * D + 4 * a + g];
      }
    BfTab<NS> nuS[D][NGP], nmS[D][NGP];
    if constexpr (NS > 0) {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int sg = 0; sg < NGP; ++sg) {
          nuS[a][sg] = bf_steps<NS>(nuB[a], 4 * sg);
          nmS[a][sg] = bf_steps<NS>(nmB[a], 4 * sg);
        }
    }
    // projection moments of [[u]] and [[mu]]
    T cu[D][C::NFJT][4], cm[D][C::NFJT][4];
#pragma unroll
    for (int jt = 0; jt < C::NFJT; ++jt) {
      V ro[D], rn[D], so[D], sn[D];
#pragma unroll
      for (int a = 0; a < D; ++a) { ro[a] = vz<V>(); rn[a] = vz<V>(); so[a] = vz<V>(); sn[a] = vz<V>(); }
      if constexpr (NS == 0) {
#pragma unroll
        for (int kk = 0; kk < C::NPK; ++kk) {
          const T ao = tb.fac_K[((f * C::NFJT + jt) * C::NPK + kk) * 64 + lane];
          const T an = tb.fac_K[((fp * C::NFJT + jt) * C::NPK + kk) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            ro[a] = M::mma(ao, uB[a][kk], ro[a]);
            rn[a] = M::mma(an, nuB[a][kk], rn[a]);
            so[a] = M::mma(ao, mB[a][kk], so[a]);
            sn[a] = M::mma(an, nmB[a][kk], sn[a]);
          }
        }
      } else {
#pragma unroll
        for (int sg = 0; sg < NGP; ++sg) {
          const BfTab<NS> ao = tb.fac_K[((f * C::NFJT + jt) * NGP + sg) * 64 + lane];
          const BfTab<NS> an = tb.fac_K[((fp * C::NFJT + jt) * NGP + sg) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            ro[a] = mma_bf<NS>(ao, uS[a][sg], ro[a]);
            rn[a] = mma_bf<NS>(an, nuS[a][sg], rn[a]);
            so[a] = mma_bf<NS>(ao, mS[a][sg], so[a]);
            sn[a] = mma_bf<NS>(an, nmS[a][sg], sn[a]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = 16 * jt + M::row(i, g);
        const bool keep = j < C::NF && tb.psi_deg[j < C::NF ? j : 0] <= lf;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s1 = 0, s2 = 0;
#pragma unroll
          for (int bb = 0; bb < D; ++bb) {
            s1 += J[a][bb] * (double)ro[bb][i] * idet - Jn[a][bb] * (double)rn[bb][i] * idetn;
            s2 += J[a][bb] * (double)so[bb][i] * idet - Jn[a][bb] * (double)sn[bb][i] * idetn;
          }
          cu[a][jt][i] = keep ? (T)s1 : (T)0;
          cm[a][jt][i] = keep ? (T)s2 : (T)0;
        }
      }
    }
    V c2[D][C::NFJT];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int jt = 0; jt < C::NFJT; ++jt) c2[a][jt] = vz<V>();
#pragma unroll 1
    for (int qt = 0; qt < C::NQFT; ++qt) {
      V to[D], tn[D], mo[D], mn[D], pu[D], pm[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        to[a] = vz<V>(); tn[a] = vz<V>(); mo[a] = vz<V>(); mn[a] = vz<V>(); pu[a] = vz<V>(); pm[a] = vz<V>();
      }
      if constexpr (NS == 0) {
#pragma unroll
        for (int kk = 0; kk < C::NPK; ++kk) {
          const T ao = tb.fac_Tr[((f * C::NQFT + qt) * C::NPK + kk) * 64 + lane];
          const T an = tb.fac_Tr[((fp * C::NQFT + qt) * C::NPK + kk) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            to[a] = M::mma(ao, uB[a][kk], to[a]);
            tn[a] = M::mma(an, nuB[a][kk], tn[a]);
            mo[a] = M::mma(ao, mB[a][kk], mo[a]);
            mn[a] = M::mma(an, nmB[a][kk], mn[a]);
          }
        }
#pragma unroll
        for (int jk = 0; jk < C::NFK; ++jk) {
          const T ap = tb.fac_Psi[(qt * C::NFK + jk) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            pu[a] = M::mma(ap, cu[a][jk / 4][jk % 4], pu[a]);
            pm[a] = M::mma(ap, cm[a][jk / 4][jk % 4], pm[a]);
          }
        }
      } else {
#pragma unroll
        for (int sg = 0; sg < NGP; ++sg) {
          const BfTab<NS> ao = tb.fac_Tr[((f * C::NQFT + qt) * NGP + sg) * 64 + lane];
          const BfTab<NS> an = tb.fac_Tr[((fp * C::NQFT + qt) * NGP + sg) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            to[a] = mma_bf<NS>(ao, uS[a][sg], to[a]);
            tn[a] = mma_bf<NS>(an, nuS[a][sg], tn[a]);
            mo[a] = mma_bf<NS>(ao, mS[a][sg], mo[a]);
            mn[a] = mma_bf<NS>(an, nmS[a][sg], mn[a]);
          }
        }
        // steps jk = 4 jt + i of the moments: group jt holds c[.][jt][0..3]
#pragma unroll
        for (int jt = 0; jt < C::NFJT; ++jt) {
          const BfTab<NS> ap = tb.fac_Psi[(qt * C::NFJT + jt) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            pu[a] = mma_bf<NS>(ap, bf_split4<NS>(cu[a][jt][0], cu[a][jt][1], cu[a][jt][2], cu[a][jt][3]), pu[a]);
            pm[a] = mma_bf<NS>(ap, bf_split4<NS>(cm[a][jt][0], cm[a][jt][1], cm[a][jt][2], cm[a][jt][3]), pm[a]);
          }
        }
      }
      // reduced forms: u.n at this tile's points from the facet DoFs
      // (register i: the point of this lane's row i)
      constexpr bool UN_DOF = !std::is_same_v<T, double>;
      d4 un4 = vz<d4>();
      if constexpr (UN_DOF) {
#pragma unroll
        for (int jk = 0; jk < C::NFK; ++jk)
          un4 = VM<double>::mma(psi_n[(qt * C::NFK + jk) * 64 + lane], xF[jk], un4);
      }
      T h[D][4], aw[D][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 16 * qt + M::row(i, g);
        const double wq = q < C::NQF ? tb.wf[q] : 0.0;
        double uo[D], un[D], mo2[D], mn2[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
          for (int bb = 0; bb < D; ++bb) {
            s1 += J[a][bb] * (double)to[bb][i];
            s2 += Jn[a][bb] * (double)tn[bb][i];
            s3 += J[a][bb] * (double)mo[bb][i];
            s4 += Jn[a][bb] * (double)mn[bb][i];
          }
          uo[a] = s1 * idet; un[a] = s2 * idetn; mo2[a] = s3 * idet; mn2[a] = s4 * idetn;
        }
        double unn = 0;
        if constexpr (UN_DOF) {
          unn = un4[i];
        } else {
#pragma unroll
          for (int a = 0; a < D; ++a) unn += 0.5 * (uo[a] + un[a]) * nrm[a];
        }
        double s_avg = 0, s_up = 0, jm[D], jmp[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          jm[a] = mo2[a] - mn2[a];
          jmp[a] = jm[a] - (double)pm[a][i];
          const double jup = (uo[a] - un[a]) - (double)pu[a][i];
          s_avg += 0.5 * (uo[a] + un[a]) * jm[a];
          s_up += jup * jmp[a];
        }
        // sgn(0) := 0, u.n within 1e-8 |<u>| of zero counting as zero (a
        // field tangential to the facet gives u.n as rounding noise; two
        // FP64 evaluations of u.n differ by up to about 1e-11 |<u>|)
        double aa = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) aa += 0.25 * (uo[a] + un[a]) * (uo[a] + un[a]);
        const double sg = fabs(unn) <= 1e-8 * sqrt(aa) ? 0.0 : (unn > 0 ? 1.0 : -1.0);
        const double s = s_avg + 0.5 * sg * s_up;
        const double hu = 0.5 * fabs(unn);
        double gg[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double av_ = hu * jmp[a];
          aw[a][i] = (T)av_;
          gg[a] = 0.5 * s * nrm[a] + 0.5 * unn * jm[a] + av_;
        }
        const double sh = wq * nfn * idet;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double t2 = 0;
#pragma unroll
          for (int bb = 0; bb < D; ++bb) t2 += J[bb][a] * gg[bb];
          h[a][i] = (T)(t2 * sh);
        }
      }
      V t[D][C::NAT];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int at = 0; at < C::NAT; ++at) t[a][at] = vz<V>();
      if constexpr (NS == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int at = 0; at < C::NAT; ++at) {
            const T av = tb.fac_TrT[(((f * C::NQFT + qt) * 4 + i) * C::NAT + at) * 64 + lane];
#pragma unroll
            for (int a = 0; a < D; ++a) t[a][at] = M::mma(av, h[a][i], t[a][at]);
          }
      } else {
        BfTab<NS> hb[D];
#pragma unroll
        for (int a = 0; a < D; ++a) hb[a] = bf_split4<NS>(h[a][0], h[a][1], h[a][2], h[a][3]);
#pragma unroll
        for (int at = 0; at < C::NAT; ++at) {
          const BfTab<NS> av = tb.fac_TrT[((f * C::NQFT + qt) * C::NAT + at) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) t[a][at] = mma_bf<NS>(av, hb[a], t[a][at]);
        }
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int at = 0; at < C::NAT; ++at)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[a][at][i] += (double)t[a][at][i];
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
    V t[D][C::NAT];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < C::NAT; ++at) t[a][at] = vz<V>();
    if constexpr (NS == 0) {
#pragma unroll
      for (int jk = 0; jk < C::NFK; ++jk)
#pragma unroll
        for (int at = 0; at < C::NAT; ++at) {
          const T av = tb.fac_KT[((f * C::NAT + at) * C::NFK + jk) * 64 + lane];
#pragma unroll
          for (int a = 0; a < D; ++a) t[a][at] = M::mma(av, cc[a][jk / 4][jk % 4], t[a][at]);
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
          for (int a = 0; a < D; ++a) t[a][at] = mma_bf<NS>(av, cb[a], t[a][at]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < C::NAT; ++at)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[a][at][i] += (double)t[a][at][i];
  }

  // dual transform in FP64 for every form, from the FP64 sums: the dual
  // basis' condition number grows quickly with k (about 4e5 at k = 5 in 3D)
  const int64_t off = mesh.F * C::NF;
  const double* const dual = dual_f64(tb);
#pragma unroll
  for (int jt = 0; jt < C::NJT; ++jt) {
    d4 o = vz<d4>();
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int at = 0; at < C::NAT; ++at)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          o = VM<double>::mma(dual[((((jt * D + a) * C::NAT + at) * 4) + i) * 64 + lane], acc[a][at][i], o);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = 16 * jt + VM<double>::row(i, g);
      if (valid && j < C::N) {
        if (j < C::NFL) oslot[ee * C::NFL + j] = (double)o[i] * Gr[GEO_NFN + j / C::NF];
        else out[off + ee * C::NINT + (j - C::NFL)] = (double)o[i] * Gr[GEO_SI];
      }
    }
  }
}

template <typename T, int D, int KK>
void launch_vjp(hipStream_t s, const T* mu_u, const T* mu_mu, double* out, double* slot, const DevMesh& mesh,
                const DevTables<T>& tb, const double* udual, const double* psi_n) {
  HOPU_LAUNCH((k_vjp<T, D, KK>), dim3((unsigned)mesh.nb), dim3(64), 0, s, mu_u, mu_mu, out, slot, mesh, tb, udual,
              psi_n);
}
template <int NS, int D, int KK>
void launch_vjp_bf(hipStream_t s, const float* mu_u, const float* mu_mu, double* out, double* slot,
                   const DevMesh& mesh, const DevTables<BfPack<NS>>& tb, const double* udual, const double* psi_n) {
  HOPU_LAUNCH((k_vjp<float, D, KK, NS>), dim3((unsigned)mesh.nb), dim3(64), 0, s, mu_u, mu_mu, out, slot, mesh,
              tb, udual, psi_n);
}

#define HOPU_VJP_INST(D, KK)                                                                                  \
  template void launch_vjp<double, D, KK>(hipStream_t, const double*, const double*, double*, double*,       \
                                          const DevMesh&, const DevTables<double>&, const double*,           \
                                          const double*);                                                    \
  template void launch_vjp<float, D, KK>(hipStream_t, const float*, const float*, double*, double*,          \
                                         const DevMesh&, const DevTables<float>&, const double*,            \
                                         const double*);                                                    \
  template void launch_vjp_bf<2, D, KK>(hipStream_t, const float*, const float*, double*, double*,           \
                                        const DevMesh&, const DevTables<BfPack<2>>&, const double*,         \
                                        const double*);                                                     \
  template void launch_vjp_bf<3, D, KK>(hipStream_t, const float*, const float*, double*, double*,           \
                                        const DevMesh&, const DevTables<BfPack<3>>&, const double*,         \
                                        const double*);
HOPU_VJP_INST(2, 1)
HOPU_VJP_INST(2, 2)
HOPU_VJP_INST(2, 3)
HOPU_VJP_INST(2, 4)
HOPU_VJP_INST(3, 1)
HOPU_VJP_INST(3, 2)
HOPU_VJP_INST(3, 3)
HOPU_VJP_INST(3, 4)
HOPU_VJP_INST(3, 5)

}  // namespace hopu
