// Host-side tables and per-element frames of the implicit Stokes step
// (paper section 2.2: Sigma_h, W_h, V^_h, a_h, b_2h; section 2.3: eq.
// (MCS_step1)).  Plain C++17.
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"
#include "host_tables.hpp"
#include "stokes.hpp"

namespace hopu {

StokesDims stokes_dims(int dim, int k) {
  StokesDims s;
  s.dim = dim;
  s.k = k;
  s.nE = dim * dim - 1;
  s.nG = dim * (dim - 1) / 2;
  s.nP1 = dim_P(dim, k + 1);
  s.nPk = dim_P(dim, k);
  s.nsf = s.nE * s.nP1;
  s.nft = dim_P(dim - 1, k + 1);
  s.nf = dim_P(dim - 1, k);
  s.ntop = s.nft - s.nf;
  s.ncons = (dim + 1) * (dim - 1) * s.ntop;
  s.n1 = s.nG * s.nPk + s.ncons;
  s.n = dim * dim_P(dim, k);
  s.nint = s.n - (dim + 1) * s.nf;
  s.nh = (dim + 1) * (dim - 1) * s.nf;
  s.nx = s.n + s.nh;
  s.ng = s.n1 + s.nx;
  s.nsd = dim * s.nf;
  return s;
}

static void matrix_bases(int d, std::vector<double>& Ea, std::vector<double>& Gc) {
  Ea.clear();
  Gc.clear();
  auto push = [&](std::vector<double>& v, const double* m) { v.insert(v.end(), m, m + d * d); };
  double m[9];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      if (i == j) continue;
      for (int q = 0; q < d * d; ++q) m[q] = 0.0;
      m[i * d + j] = 1.0;
      push(Ea, m);
    }
  for (int q = 0; q < d * d; ++q) m[q] = 0.0;
  m[0] = 1.0 / std::sqrt(2.0);
  m[d + 1] = -1.0 / std::sqrt(2.0);
  push(Ea, m);
  if (d == 3) {
    for (int q = 0; q < 9; ++q) m[q] = 0.0;
    m[0] = m[4] = 1.0 / std::sqrt(6.0);
    m[8] = -2.0 / std::sqrt(6.0);
    push(Ea, m);
  }
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j) {
      for (int q = 0; q < d * d; ++q) m[q] = 0.0;
      m[i * d + j] = 1.0 / std::sqrt(2.0);
      m[j * d + i] = -1.0 / std::sqrt(2.0);
      push(Gc, m);
    }
}

bool make_stokes_tables(int dim, int k, StokesTables& t, std::string& err) {
  const StokesDims sd = stokes_dims(dim, k);
  t.sd = sd;
  matrix_bases(dim, t.Ea, t.Gc);
  DualBasis db;
  if (!make_dual_basis(dim, k, db, err)) return false;
  const int n = sd.n, nP = sd.nPk, nP1 = sd.nP1, d = dim;
  // reference dual basis phi^_j = sum_(a,alpha) Dinv[(a,alpha)][j] e_a p_alpha
  std::vector<ld> pts, w;
  simplex_rule(dim, k + 2, pts, w);
  const int nq = (int)w.size();
  std::vector<ld> pk(nP), gk(nP * dim), p1(nP1), g1(nP1 * dim);
  std::vector<ld> phi((size_t)nq * n * d, 0.0L);
  std::vector<ld> P1v((size_t)nq * nP1), P1g((size_t)nq * nP1 * d), Pkv((size_t)nq * nP);
  for (int q = 0; q < nq; ++q) {
    dubiner(dim, k, &pts[q * dim], pk.data(), gk.data());
    dubiner(dim, k + 1, &pts[q * dim], p1.data(), g1.data());
    for (int a = 0; a < nP1; ++a) {
      P1v[(size_t)q * nP1 + a] = p1[a];
      for (int r = 0; r < d; ++r) P1g[((size_t)q * nP1 + a) * d + r] = g1[a * dim + r];
    }
    for (int a = 0; a < nP; ++a) Pkv[(size_t)q * nP + a] = pk[a];
    for (int j = 0; j < n; ++j)
      for (int s = 0; s < d; ++s) {
        ld v = 0.0L;
        for (int al = 0; al < nP; ++al) v += db.Dinv[(size_t)(s * nP + al) * n + j] * pk[al];
        phi[((size_t)q * n + j) * d + s] = v;
      }
  }
  // Gram of P^{k+1}: the setup kernel takes it as c I
  const ld c0 = [&] {
    ld v = 0.0L;
    for (int q = 0; q < nq; ++q) v += w[q] * P1v[(size_t)q * nP1] * P1v[(size_t)q * nP1];
    return v;
  }();
  for (int a = 0; a < nP1; ++a)
    for (int b = 0; b < nP1; ++b) {
      ld v = 0.0L;
      for (int q = 0; q < nq; ++q) v += w[q] * P1v[(size_t)q * nP1 + a] * P1v[(size_t)q * nP1 + b];
      if (std::fabs((double)(v - (a == b ? c0 : 0.0L))) > 1e-13 * (double)c0) {
        err = "stokes tables: the P^{k+1} basis is not orthogonal with equal norms";
        return false;
      }
    }
  t.MpG.assign((size_t)nP * nP1, 0.0);
  for (int b = 0; b < nP; ++b)
    for (int a = 0; a < nP1; ++a) {
      ld v = 0.0L;
      for (int q = 0; q < nq; ++q) v += w[q] * Pkv[(size_t)q * nP + b] * P1v[(size_t)q * nP1 + a];
      t.MpG[(size_t)b * nP1 + a] = (double)v;
    }
  t.TV.assign((size_t)nP1 * n * d * d, 0.0);
  for (int a = 0; a < nP1; ++a)
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < d; ++r)
        for (int s = 0; s < d; ++s) {
          ld v = 0.0L;
          for (int q = 0; q < nq; ++q)
            v += w[q] * P1g[((size_t)q * nP1 + a) * d + r] * phi[((size_t)q * n + i) * d + s];
          t.TV[(((size_t)a * n + i) * d + r) * d + s] = (double)v;
        }
  t.Mref.assign((size_t)n * n * d * d, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int r = 0; r < d; ++r)
        for (int s = 0; s < d; ++s) {
          ld v = 0.0L;
          for (int q = 0; q < nq; ++q) v += w[q] * phi[((size_t)q * n + i) * d + r] * phi[((size_t)q * n + j) * d + s];
          t.Mref[(((size_t)i * n + j) * d + r) * d + s] = (double)v;
        }
  // facet moments of p_alpha (P^{k+1}) against psi_m (P^{k+1}(F))
  std::vector<ld> sp, sw;
  simplex_rule(dim - 1, k + 2, sp, sw);
  const int ns = (int)sw.size();
  t.Phi.assign((size_t)(dim + 1) * nP1 * sd.nft, 0.0);
  std::vector<ld> psi(sd.nft);
  for (int f = 0; f <= dim; ++f) {
    ld o[3], Em[6], N[3];
    ref_facet(dim, f, o, Em, N);
    for (int q = 0; q < ns; ++q) {
      ld x[3];
      for (int a = 0; a < dim; ++a) {
        x[a] = o[a];
        for (int c = 0; c < dim - 1; ++c) x[a] += Em[a * (dim - 1) + c] * sp[q * (dim - 1) + c];
      }
      dubiner(dim, k + 1, x, p1.data(), g1.data());
      facet_psi(dim, k + 1, &sp[q * (dim - 1)], psi.data());
      for (int a = 0; a < nP1; ++a)
        for (int m = 0; m < sd.nft; ++m)
          t.Phi[((size_t)f * nP1 + a) * sd.nft + m] += (double)(sw[q] * p1[a] * psi[m]);
    }
  }
  // the kernel's D = -c0 |det J| / (2 nu) I: fold c0 into the tables' use
  // by scaling MpG, TV, Phi by 1/sqrt(c0) (sigma's coefficients rescale; S_T
  // does not change)
  const double isc = 1.0 / std::sqrt((double)c0);
  for (auto& v : t.MpG) v *= isc;
  for (auto& v : t.TV) v *= isc;
  for (auto& v : t.Phi) v *= isc;
  return true;
}

void make_stokes_geometry(int dim, int64_t E, const std::vector<double>& xyz, const std::vector<double>& geo,
                          const std::vector<int32_t>& fid, std::vector<double>& out) {
  const int dp1 = dim + 1;
  out.assign((size_t)E * STG, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    const double* g = &geo[(size_t)e * GEO_STRIDE];
    const double* x = &xyz[(size_t)e * dp1 * dim];
    double* o = &out[(size_t)e * STG];
    double J[9] = {0}, Ji[9] = {0};
    for (int r = 0; r < dim; ++r)
      for (int c = 0; c < dim; ++c) J[r * 3 + c] = g[r * dim + c];
    const double det = g[GEO_DET];
    if (dim == 2) {
      Ji[0] = J[4] / det; Ji[1] = -J[1] / det;
      Ji[3] = -J[3] / det; Ji[4] = J[0] / det;
    } else {
      Ji[0] = (J[4] * J[8] - J[5] * J[7]) / det;
      Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
      Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
      Ji[3] = (J[5] * J[6] - J[3] * J[8]) / det;
      Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
      Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
      Ji[6] = (J[3] * J[7] - J[4] * J[6]) / det;
      Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
      Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    }
    for (int q = 0; q < 9; ++q) { o[q] = J[q]; o[9 + q] = Ji[q]; }
    o[18] = det;
    for (int f = 0; f < dp1; ++f) {
      double* fr = o + 20 + 11 * f;
      const double sgn = ((f % 2) ? -1.0 : 1.0) * (det > 0 ? 1.0 : -1.0);
      double nout[3] = {0, 0, 0}, nF[3] = {0, 0, 0}, t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) {
        nout[a] = g[GEO_NRM + f * dim + a];
        nF[a] = sgn * nout[a];
      }
      int lv[3], c = 0;
      for (int v = 0; v < dp1; ++v) if (v != f) lv[c++] = v;
      double nn = 0.0;
      for (int a = 0; a < dim; ++a) {
        t1[a] = x[lv[1] * dim + a] - x[lv[0] * dim + a];
        nn += t1[a] * t1[a];
      }
      nn = std::sqrt(nn);
      for (int a = 0; a < dim; ++a) t1[a] /= nn;
      if (dim == 3) {
        t2[0] = nF[1] * t1[2] - nF[2] * t1[1];
        t2[1] = nF[2] * t1[0] - nF[0] * t1[2];
        t2[2] = nF[0] * t1[1] - nF[1] * t1[0];
      }
      for (int a = 0; a < 3; ++a) { fr[a] = nout[a]; fr[3 + a] = t1[a]; fr[6 + a] = t2[a]; }
      fr[9] = g[GEO_NFN + f];
      fr[10] = fid[(size_t)e * dp1 + f] >= 0 ? 1.0 : 0.0;
    }
  }
}

}  // namespace hopu
