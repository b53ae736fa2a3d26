// Host precompute: quadrature, dual basis, tables, topology, geometry.
#include "host_tables.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

namespace hopu {

int dim_P(int dim, int k) {
  if (k < 0) return 0;
  if (dim == 1) return k + 1;
  if (dim == 2) return (k + 1) * (k + 2) / 2;
  return (k + 1) * (k + 2) * (k + 3) / 6;
}

static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

Sizes make_sizes(int dim, int k) {
  Sizes s;
  s.dim = dim; s.k = k;
  s.nP = dim_P(dim, k);
  s.nPs = (s.nP + 3) / 4 * 4;
  s.nm = dim * s.nPs;
  s.n = dim * s.nP;
  s.nf = dim_P(dim - 1, k);
  s.nfl = (dim + 1) * s.nf;
  s.nint = s.n - s.nfl;
  s.pv = (3 * k + 1) / 2;       // ceil(3k/2): degree 3k-1 exact
  s.pf = (3 * k + 2) / 2;       // ceil((3k+1)/2): degree 3k exact
  s.nqv = ipow(s.pv, dim);
  s.nqf = ipow(s.pf, dim - 1);
  return s;
}

// ------------------------------------------------------------ Jacobi
// P_n^{(a,b)}(x) by the three-term recurrence; also returns P_{n-1}.
static ld jacobi(int n, ld a, ld b, ld x) {
  if (n == 0) return 1.0L;
  ld p0 = 1.0L, p1 = 0.5L * ((a + b + 2.0L) * x + a - b);
  for (int m = 1; m < n; ++m) {
    ld c = 2.0L * m + a + b;
    ld a1 = 2.0L * (m + 1) * (m + a + b + 1) * c;
    ld a2 = (c + 1.0L) * (a * a - b * b);
    ld a3 = c * (c + 1.0L) * (c + 2.0L);
    ld a4 = 2.0L * (m + a) * (m + b) * (c + 2.0L);
    ld p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1; p1 = p2;
  }
  return p1;
}
static ld djacobi(int n, ld a, ld b, ld x) {
  if (n == 0) return 0.0L;
  return 0.5L * (n + a + b + 1.0L) * jacobi(n - 1, a + 1.0L, b + 1.0L, x);
}

void gauss_jacobi(int n, ld a, ld b, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(n, 0.0L);
  w.assign(n, 0.0L);
  const ld pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < n; ++i) {
    ld r = -cosl((2.0L * i + 1.0L) * pi / (2.0L * n));
    if (i > 0) r = 0.5L * (r + x[i - 1]);
    for (int it = 0; it < 200; ++it) {
      ld p = jacobi(n, a, b, r), dp = djacobi(n, a, b, r);
      ld s = 0.0L;
      for (int j = 0; j < i; ++j) s += 1.0L / (r - x[j]);
      ld delta = -p / (dp - s * p);
      r += delta;
      if (fabsl(delta) < 1e-19L) break;
    }
    x[i] = r;
  }
  std::sort(x.begin(), x.end());
  ld c = powl(2.0L, a + b + 1.0L) * expl(lgammal(n + a + 1.0L) + lgammal(n + b + 1.0L) -
                                         lgammal(n + 1.0L) - lgammal(n + a + b + 1.0L));
  for (int i = 0; i < n; ++i) {
    ld dp = djacobi(n, a, b, x[i]);
    w[i] = c / ((1.0L - x[i] * x[i]) * dp * dp);
  }
}

void simplex_rule(int dim, int npd, std::vector<ld>& pts, std::vector<ld>& w) {
  std::vector<ld> xa, wa, xb, wb, xc, wc;
  gauss_jacobi(npd, 0.0L, 0.0L, xa, wa);
  pts.clear(); w.clear();
  if (dim == 1) {
    for (int i = 0; i < npd; ++i) { pts.push_back(0.5L * (1.0L + xa[i])); w.push_back(0.5L * wa[i]); }
    return;
  }
  gauss_jacobi(npd, 1.0L, 0.0L, xb, wb);
  if (dim == 2) {
    for (int i = 0; i < npd; ++i)
      for (int j = 0; j < npd; ++j) {
        pts.push_back((1.0L + xa[i]) * (1.0L - xb[j]) / 4.0L);
        pts.push_back((1.0L + xb[j]) / 2.0L);
        w.push_back(wa[i] * wb[j] / 8.0L);
      }
    return;
  }
  gauss_jacobi(npd, 2.0L, 0.0L, xc, wc);
  for (int i = 0; i < npd; ++i)
    for (int j = 0; j < npd; ++j)
      for (int l = 0; l < npd; ++l) {
        pts.push_back((1.0L + xa[i]) * (1.0L - xb[j]) * (1.0L - xc[l]) / 8.0L);
        pts.push_back((1.0L + xb[j]) * (1.0L - xc[l]) / 4.0L);
        pts.push_back((1.0L + xc[l]) / 2.0L);
        w.push_back(wa[i] * wb[j] * wc[l] / 64.0L);
      }
}

// ------------------------------------------------------------ Dubiner
// F(x, t) = t^i P_i^{(a,0)}(2x/t - 1) with dF/dx, dF/dt (polynomial form).
static void collapsed(int i, ld a, ld x, ld t, ld& F, ld& Fx, ld& Ft) {
  ld eta = 2.0L * x / t - 1.0L;
  ld P = jacobi(i, a, 0.0L, eta), dP = djacobi(i, a, 0.0L, eta);
  F = powl(t, i) * P;
  if (i == 0) { Fx = 0.0L; Ft = 0.0L; return; }
  ld tp = powl(t, i - 1);
  Fx = tp * 2.0L * dP;
  Ft = tp * (i * P - (1.0L + eta) * dP);
}

void dubiner(int dim, int k, const ld* x, ld* val, ld* grad) {
  int m = 0;
  if (dim == 2) {
    ld t = 1.0L - x[1];
    for (int i = 0; i <= k; ++i)
      for (int j = 0; i + j <= k; ++j, ++m) {
        ld c = sqrtl(2.0L * (2 * i + 1) * (i + j + 1));
        ld A, Ax, At;
        collapsed(i, 0.0L, x[0], t, A, Ax, At);
        ld e2 = 2.0L * x[1] - 1.0L;
        ld Bv = jacobi(j, 2.0L * i + 1.0L, 0.0L, e2);
        ld dB = 2.0L * djacobi(j, 2.0L * i + 1.0L, 0.0L, e2);
        val[m] = c * A * Bv;
        grad[m * 2 + 0] = c * Ax * Bv;
        grad[m * 2 + 1] = c * (-At * Bv + A * dB);
      }
    return;
  }
  ld t = 1.0L - x[1] - x[2], s = 1.0L - x[2];
  for (int i = 0; i <= k; ++i)
    for (int j = 0; i + j <= k; ++j)
      for (int l = 0; i + j + l <= k; ++l, ++m) {
        ld c = sqrtl((2.0L * i + 1) * (2.0L * i + 2 * j + 2) * (2.0L * i + 2 * j + 2 * l + 3));
        ld A, Ax, At, Bv, Bx, Bs;
        collapsed(i, 0.0L, x[0], t, A, Ax, At);
        collapsed(j, 2.0L * i + 1.0L, x[1], s, Bv, Bx, Bs);
        ld a3 = 2.0L * i + 2.0L * j + 2.0L, e3 = 2.0L * x[2] - 1.0L;
        ld Cv = jacobi(l, a3, 0.0L, e3), dC = 2.0L * djacobi(l, a3, 0.0L, e3);
        val[m] = c * A * Bv * Cv;
        grad[m * 3 + 0] = c * Ax * Bv * Cv;
        grad[m * 3 + 1] = c * (-At * Bv * Cv + A * Bx * Cv);
        grad[m * 3 + 2] = c * (-At * Bv * Cv - A * Bs * Cv + A * Bv * dC);
      }
}

std::vector<int> facet_psi_degree(int dim, int k) {
  std::vector<int> d;
  if (dim == 2) { for (int j = 0; j <= k; ++j) d.push_back(j); return d; }
  for (int m = 0; m <= k; ++m) for (int q = 0; q <= m; ++q) d.push_back(m);
  return d;
}

void facet_psi(int dim, int k, const ld* s, ld* out) {
  if (dim == 2) {
    for (int j = 0; j <= k; ++j) out[j] = sqrtl(2.0L * j + 1.0L) * jacobi(j, 0, 0, 2.0L * s[0] - 1.0L);
    return;
  }
  int idx = 0;
  ld t = 1.0L - s[1];
  for (int m = 0; m <= k; ++m)
    for (int q = 0; q <= m; ++q, ++idx) {
      int p = m - q;
      ld A, Ax, At;
      collapsed(p, 0.0L, s[0], t, A, Ax, At);
      ld c = sqrtl(2.0L * (2 * p + 1) * (p + q + 1));
      out[idx] = c * A * jacobi(q, 2.0L * p + 1.0L, 0.0L, 2.0L * s[1] - 1.0L);
    }
}

// graded lex: degree ascending, then descending lexicographic
static std::vector<std::array<int, 3>> multi_indices(int dim, int kmin, int kmax) {
  std::vector<std::array<int, 3>> out;
  for (int deg = kmin; deg <= kmax; ++deg) {
    std::vector<std::array<int, 3>> lvl;
    if (dim == 2) {
      for (int a = deg; a >= 0; --a) lvl.push_back({a, deg - a, 0});
    } else {
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) lvl.push_back({a, b, deg - a - b});
    }
    out.insert(out.end(), lvl.begin(), lvl.end());
  }
  return out;
}

void interior_tests(int dim, int k, const ld* x, ld* out) {
  ld xt[3];
  for (int a = 0; a < dim; ++a) xt[a] = x[a] - 1.0L / (dim + 1);
  auto mono = [&](const std::array<int, 3>& e) {
    ld v = 1.0L;
    for (int a = 0; a < dim; ++a) v *= powl(xt[a], e[a]);
    return v;
  };
  int m = 0;
  for (auto beta : multi_indices(dim, 1, k - 1)) {
    for (int a = 0; a < dim; ++a) {
      if (beta[a] == 0) { out[m * dim + a] = 0.0L; continue; }
      auto e = beta; e[a] -= 1;
      out[m * dim + a] = beta[a] * mono(e);
    }
    ++m;
  }
  if (k < 2) return;
  auto betas = multi_indices(dim, 0, k - 2);
  if (dim == 2) {
    for (auto beta : betas) {
      ld v = mono(beta);
      out[m * 2 + 0] = -xt[1] * v;
      out[m * 2 + 1] = xt[0] * v;
      ++m;
    }
    return;
  }
  for (int i = 0; i < 3; ++i)
    for (auto beta : betas) {
      if (i == 0 && beta[0] >= 1) continue;
      ld v = mono(beta);
      // x~ x (e_i v)
      ld e[3] = {0, 0, 0};
      e[i] = v;
      out[m * 3 + 0] = xt[1] * e[2] - xt[2] * e[1];
      out[m * 3 + 1] = xt[2] * e[0] - xt[0] * e[2];
      out[m * 3 + 2] = xt[0] * e[1] - xt[1] * e[0];
      ++m;
    }
}

void ref_facet(int dim, int i, ld* o, ld* E, ld* N) {
  ld V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  int lv[3], c = 0;
  for (int v = 0; v <= dim; ++v) if (v != i) lv[c++] = v;
  for (int a = 0; a < dim; ++a) o[a] = V[lv[0]][a];
  for (int j = 0; j < dim - 1; ++j)
    for (int a = 0; a < dim; ++a) E[a * (dim - 1) + j] = V[lv[j + 1]][a] - V[lv[0]][a];
  if (dim == 2) {
    N[0] = E[1 * 1 + 0];
    N[1] = -E[0 * 1 + 0];
  } else {
    ld t1[3] = {E[0], E[2], E[4]}, t2[3] = {E[1], E[3], E[5]};
    N[0] = t1[1] * t2[2] - t1[2] * t2[1];
    N[1] = t1[2] * t2[0] - t1[0] * t2[2];
    N[2] = t1[0] * t2[1] - t1[1] * t2[0];
  }
}

static bool invert(int n, const std::vector<ld>& A, std::vector<ld>& Ai) {
  std::vector<ld> M(A);
  Ai.assign(n * n, 0.0L);
  for (int i = 0; i < n; ++i) Ai[i * n + i] = 1.0L;
  // row equilibration first (the interior functionals have small norms)
  for (int i = 0; i < n; ++i) {
    ld s = 0;
    for (int j = 0; j < n; ++j) s = std::max(s, fabsl(M[i * n + j]));
    if (s == 0) return false;
    for (int j = 0; j < n; ++j) { M[i * n + j] /= s; Ai[i * n + j] /= s; }
  }
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r) if (fabsl(M[r * n + c]) > fabsl(M[p * n + c])) p = r;
    if (M[p * n + c] == 0) return false;
    if (p != c)
      for (int j = 0; j < n; ++j) { std::swap(M[p * n + j], M[c * n + j]); std::swap(Ai[p * n + j], Ai[c * n + j]); }
    ld d = M[c * n + c];
    for (int j = 0; j < n; ++j) { M[c * n + j] /= d; Ai[c * n + j] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      ld f = M[r * n + c];
      if (f == 0) continue;
      for (int j = 0; j < n; ++j) { M[r * n + j] -= f * M[c * n + j]; Ai[r * n + j] -= f * Ai[c * n + j]; }
    }
  }
  return true;
}

bool make_dual_basis(int dim, int k, DualBasis& out, std::string& err) {
  Sizes s = make_sizes(dim, k);
  out.sz = s;
  int n = s.n, nP = s.nP, nf = s.nf;
  out.D.assign(n * n, 0.0L);
  std::vector<ld> sp, sw, vp, vw;
  simplex_rule(dim - 1, k + 2, sp, sw);
  simplex_rule(dim, k + 2, vp, vw);
  std::vector<ld> val(nP), grad(nP * dim), psi(nf), q(std::max(1, s.nint) * dim);
  for (int i = 0; i <= dim; ++i) {
    ld o[3], E[6], N[3];
    ref_facet(dim, i, o, E, N);
    for (size_t qq = 0; qq < sw.size(); ++qq) {
      const ld* sq = &sp[qq * (dim - 1)];
      ld x[3];
      for (int a = 0; a < dim; ++a) {
        x[a] = o[a];
        for (int j = 0; j < dim - 1; ++j) x[a] += E[a * (dim - 1) + j] * sq[j];
      }
      dubiner(dim, k, x, val.data(), grad.data());
      facet_psi(dim, k, sq, psi.data());
      for (int jj = 0; jj < nf; ++jj)
        for (int a = 0; a < dim; ++a)
          for (int al = 0; al < nP; ++al)
            out.D[(i * nf + jj) * n + a * nP + al] += sw[qq] * psi[jj] * val[al] * N[a];
    }
  }
  for (size_t qq = 0; qq < vw.size(); ++qq) {
    const ld* x = &vp[qq * dim];
    dubiner(dim, k, x, val.data(), grad.data());
    if (s.nint > 0) interior_tests(dim, k, x, q.data());
    for (int m = 0; m < s.nint; ++m)
      for (int a = 0; a < dim; ++a)
        for (int al = 0; al < nP; ++al)
          out.D[(s.nfl + m) * n + a * nP + al] += vw[qq] * q[m * dim + a] * val[al];
  }
  if (!invert(n, out.D, out.Dinv)) { err = "singular DoF matrix"; return false; }
  return true;
}

bool make_ref_tables(int dim, int k, RefTables& t, std::string& err) {
  DualBasis db;
  if (!make_dual_basis(dim, k, db, err)) return false;
  Sizes s = db.sz;
  t.sz = s;
  int nP = s.nP, nf = s.nf;
  std::vector<ld> vp, vw, sp, sw;
  simplex_rule(dim, s.pv, vp, vw);
  simplex_rule(dim - 1, s.pf, sp, sw);
  t.wv.assign(vw.begin(), vw.end());
  t.wf.assign(sw.begin(), sw.end());
  t.xv.assign(vp.begin(), vp.end());
  t.sf.assign(sp.begin(), sp.end());
  std::vector<ld> val(nP), grad(nP * dim), psi(nf);
  t.V.resize(s.nqv * nP);
  t.dV.resize(s.nqv * nP * dim);
  for (int q = 0; q < s.nqv; ++q) {
    dubiner(dim, k, &vp[q * dim], val.data(), grad.data());
    for (int al = 0; al < nP; ++al) {
      t.V[q * nP + al] = (double)val[al];
      for (int b = 0; b < dim; ++b) t.dV[(q * nP + al) * dim + b] = (double)grad[al * dim + b];
    }
  }
  t.Psi.resize(s.nqf * nf);
  t.psi_deg = facet_psi_degree(dim, k);
  std::vector<ld> psiq(s.nqf * nf);
  for (int q = 0; q < s.nqf; ++q) {
    facet_psi(dim, k, &sp[q * (dim - 1)], psi.data());
    for (int j = 0; j < nf; ++j) { psiq[q * nf + j] = psi[j]; t.Psi[q * nf + j] = (double)psi[j]; }
  }
  t.Tr.resize((dim + 1) * s.nqf * nP);
  t.Kf.assign((dim + 1) * nf * nP, 0.0);
  for (int f = 0; f <= dim; ++f) {
    ld o[3], E[6], N[3];
    ref_facet(dim, f, o, E, N);
    std::vector<ld> K(nf * nP, 0.0L);
    for (int q = 0; q < s.nqf; ++q) {
      ld x[3];
      for (int a = 0; a < dim; ++a) {
        x[a] = o[a];
        for (int j = 0; j < dim - 1; ++j) x[a] += E[a * (dim - 1) + j] * sp[q * (dim - 1) + j];
      }
      dubiner(dim, k, x, val.data(), grad.data());
      for (int al = 0; al < nP; ++al) t.Tr[(f * s.nqf + q) * nP + al] = (double)val[al];
      for (int j = 0; j < nf; ++j)
        for (int al = 0; al < nP; ++al) K[j * nP + al] += sw[q] * psiq[q * nf + j] * val[al];
    }
    for (int i = 0; i < nf * nP; ++i) t.Kf[f * nf * nP + i] = (double)K[i];
  }
  t.D.assign(db.D.begin(), db.D.end());
  t.Dinv.assign(db.Dinv.begin(), db.Dinv.end());
  // projection: divergence moments of the modal basis against P^{k-1}
  // (the volume rule integrates degree 2k-2 exactly)
  {
    const int nQ = dim_P(dim, k - 1);
    t.nQ = nQ;
    t.Bm.assign((size_t)nQ * s.nm, 0.0);
    std::vector<ld> qv(nQ), qg(nQ * dim);
    std::vector<ld> acc((size_t)nQ * s.nm, 0.0L);
    for (int q = 0; q < s.nqv; ++q) {
      dubiner(dim, k, &vp[q * dim], val.data(), grad.data());
      dubiner(dim, k - 1, &vp[q * dim], qv.data(), qg.data());
      for (int be = 0; be < nQ; ++be)
        for (int a = 0; a < dim; ++a)
          for (int al = 0; al < nP; ++al)
            acc[(size_t)be * s.nm + modal_row(dim, a, al)] += vw[q] * grad[al * dim + a] * qv[be];
    }
    for (size_t i = 0; i < acc.size(); ++i) t.Bm[i] = (double)acc[i];
  }
  return true;
}

FragDims frag_dims(const Sizes& s) {
  FragDims d;
  d.NMT = (s.nm + 15) / 16;
  d.NK = (s.n + 3) / 4;
  d.NQVT = (s.nqv + 15) / 16;
  d.NPK = s.nPs / 4;
  d.NAT = (s.nP + 15) / 16;
  d.NQFT = (s.nqf + 15) / 16;
  d.NFJT = (s.nf + 15) / 16;
  d.NFK = 4 * d.NFJT;
  d.NJT = (s.n + 15) / 16;
  d.NMQ = 4 * d.NMT;
  return d;
}

std::vector<uint16_t> split_bf16_table(const std::vector<double>& t, int outer, int nsteps, int inner, int ns) {
  const int ng = (nsteps + 3) / 4;
  std::vector<uint16_t> out((size_t)outer * ng * inner * 64 * ns * 4, 0);
  for (int o = 0; o < outer; ++o)
    for (int sg = 0; sg < ng; ++sg)
      for (int in = 0; in < inner; ++in)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 4; ++j) {
            const int st = 4 * sg + j;
            if (st >= nsteps) continue;
            float r = (float)t[(((size_t)o * nsteps + st) * inner + in) * 64 + l];
            uint16_t* dst = &out[((((size_t)o * ng + sg) * inner + in) * 64 + l) * ns * 4];
            for (int term = 0; term < ns; ++term) {
              uint32_t u;
              std::memcpy(&u, &r, 4);
              const uint32_t h = u & 0xFFFF0000u;
              float hv;
              std::memcpy(&hv, &h, 4);
              dst[term * 4 + j] = (uint16_t)(h >> 16);
              r -= hv;
            }
          }
  return out;
}

void make_bf16_tables(const FragTables& f, const Sizes& s, int ns, BfTables& b) {
  const FragDims d = frag_dims(s);
  const int nfc = s.dim + 1;
  b.vol_V = split_bf16_table(f.vol_V, d.NQVT, d.NPK, 1, ns);
  b.vol_dVT = split_bf16_table(f.vol_dVT, d.NQVT, 4, s.dim * d.NAT, ns);
  b.fac_Tr = split_bf16_table(f.fac_Tr, nfc * d.NQFT, d.NPK, 1, ns);
  b.fac_TrT = split_bf16_table(f.fac_TrT, nfc * d.NQFT, 4, d.NAT, ns);
  b.fac_K = split_bf16_table(f.fac_K, nfc * d.NFJT, d.NPK, 1, ns);
  b.fac_Psi = split_bf16_table(f.fac_Psi, d.NQFT, d.NFK, 1, ns);
  b.fac_PsiT = split_bf16_table(f.fac_PsiT, d.NQFT, 4, d.NFJT, ns);
  b.fac_KT = split_bf16_table(f.fac_KT, nfc * d.NAT, d.NFK, 1, ns);
  b.vol_dV = split_bf16_table(f.vol_dV, d.NQVT * s.dim, d.NPK, 1, ns);
  b.vol_VT = split_bf16_table(f.vol_VT, d.NQVT, 4, d.NAT, ns);
}

void make_frag_tables(const RefTables& t, RowMap rm, FragTables& f) {
  const Sizes& s = t.sz;
  FragDims fd = frag_dims(s);
  const int dim = s.dim, nP = s.nP, n = s.n, nf = s.nf;
  auto rowof = [&](int i, int g) { return rm == ROWMAP_F64 ? 4 * i + g : 4 * g + i; };
  // modal row rho -> (a, alpha) or -1
  auto rho_inv = [&](int rho, int& a, int& al) {
    int blk = rho / (4 * dim), rem = rho % (4 * dim);
    a = rem / 4;
    al = 4 * blk + rem % 4;
    return (rho < s.nm && al < nP);
  };
  auto Dinv = [&](int a, int al, int j) { return t.Dinv[(a * nP + al) * n + j]; };
  auto D = [&](int j, int a, int al) { return t.D[j * n + a * nP + al]; };
  // modal: dual rows j = 4 kk + g in order
  f.modal.assign(fd.NMT * fd.NK * 64, 0.0);
  for (int mt = 0; mt < fd.NMT; ++mt)
    for (int kk = 0; kk < fd.NK; ++kk)
      for (int l = 0; l < 64; ++l) {
        int a, al, rho = 16 * mt + (l & 15), j = 4 * kk + (l >> 4);
        if (!rho_inv(rho, a, al) || j >= n) continue;
        f.modal[(mt * fd.NK + kk) * 64 + l] = Dinv(a, al, j);
      }
  // mass / preconditioner: dual rows in mass_row order.  The kernels see the
  // same layout in both precisions: register i of lane group g holds modal
  // row 16 mt + 4 i + g after the first contraction and dual step 4 jt + i
  // after the second.  Output row m of an MFMA tile sits in register m/4 of
  // group m%4 (f64) or in register m%4 of group m/4 (f32), so the tables'
  // M rows are permuted accordingly; the K side is the same for both.
  const bool f32 = rm == ROWMAP_F32;
  f.mass_in.assign(fd.NMT * fd.NK * 64, 0.0);
  f.prec_in.assign(fd.NMT * fd.NK * 64, 0.0);
  for (int mt = 0; mt < fd.NMT; ++mt)
    for (int kk = 0; kk < fd.NK; ++kk)
      for (int l = 0; l < 64; ++l) {
        const int m = l & 15;
        int a, al, rho = 16 * mt + (f32 ? 4 * (m % 4) + m / 4 : m), j = mass_row(s, kk, l >> 4);
        if (!rho_inv(rho, a, al) || j < 0) continue;
        f.mass_in[(mt * fd.NK + kk) * 64 + l] = Dinv(a, al, j);
        f.prec_in[(mt * fd.NK + kk) * 64 + l] = D(j, a, al);
      }
  f.mass_out.assign(fd.NJT * fd.NMQ * 64, 0.0);
  f.prec_out.assign(fd.NJT * fd.NMQ * 64, 0.0);
  for (int jt = 0; jt < fd.NJT; ++jt)
    for (int rq = 0; rq < fd.NMQ; ++rq)
      for (int l = 0; l < 64; ++l) {
        const int m = l & 15;
        const int step = 4 * jt + (f32 ? m % 4 : m / 4), grp = f32 ? m / 4 : m % 4;
        int j = mass_row(s, step, grp), rho = 16 * (rq / 4) + 4 * (rq % 4) + (l >> 4), a, al;
        if (j < 0 || !rho_inv(rho, a, al)) continue;
        f.mass_out[(jt * fd.NMQ + rq) * 64 + l] = Dinv(a, al, j);
        f.prec_out[(jt * fd.NMQ + rq) * 64 + l] = D(j, a, al);
      }
  // projection: Bm (rows beta, K = modal rows in the output-tile order of the
  // first contraction) and Bm^T (rows rho, K = beta in the output order of
  // the Bm contraction), f64 register layout
  {
    const int nQ = t.nQ, NBT = proj_nbt(nQ), NQK = proj_nqk(nQ);
    auto Bm = [&](int be, int rho) { return t.Bm[(size_t)be * s.nm + rho]; };
    f.proj_b.assign((size_t)NBT * fd.NMQ * 64, 0.0);
    for (int bt = 0; bt < NBT; ++bt)
      for (int rq = 0; rq < fd.NMQ; ++rq)
        for (int l = 0; l < 64; ++l) {
          const int be = 16 * bt + (l & 15), rho = 16 * (rq / 4) + rowof(rq % 4, l >> 4);
          if (be < nQ && rho < s.nm) f.proj_b[((size_t)bt * fd.NMQ + rq) * 64 + l] = Bm(be, rho);
        }
    f.proj_bt.assign((size_t)fd.NMT * NQK * 64, 0.0);
    for (int mt = 0; mt < fd.NMT; ++mt)
      for (int kk = 0; kk < NQK; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int rho = 16 * mt + (l & 15), be = 16 * (kk / 4) + rowof(kk % 4, l >> 4);
          if (be < nQ && rho < s.nm) f.proj_bt[((size_t)mt * NQK + kk) * 64 + l] = Bm(be, rho);
        }
    f.proj_kab.assign((size_t)dim * dim * nQ * nQ, 0.0);
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b)
        for (int be = 0; be < nQ; ++be)
          for (int ga = 0; ga < nQ; ++ga) {
            long double acc = 0.0L;
            for (int al = 0; al < nP; ++al)
              acc += (long double)Bm(be, modal_row(dim, a, al)) * Bm(ga, modal_row(dim, b, al));
            f.proj_kab[(((size_t)a * dim + b) * nQ + be) * nQ + ga] = (double)acc;
          }
  }
  // volume
  f.vol_V.assign(fd.NQVT * fd.NPK * 64, 0.0);
  f.vol_dV.assign(fd.NQVT * dim * fd.NPK * 64, 0.0);
  for (int qt = 0; qt < fd.NQVT; ++qt)
    for (int kk = 0; kk < fd.NPK; ++kk)
      for (int l = 0; l < 64; ++l) {
        int q = 16 * qt + (l & 15), al = 4 * kk + (l >> 4);
        if (q >= s.nqv || al >= nP) continue;
        f.vol_V[(qt * fd.NPK + kk) * 64 + l] = t.V[q * nP + al];
        for (int b = 0; b < dim; ++b)
          f.vol_dV[((qt * dim + b) * fd.NPK + kk) * 64 + l] = t.dV[(q * nP + al) * dim + b];
      }
  f.vol_dVT.assign(fd.NQVT * 4 * dim * fd.NAT * 64, 0.0);
  f.vol_VT.assign(fd.NQVT * 4 * fd.NAT * 64, 0.0);
  for (int qt = 0; qt < fd.NQVT; ++qt)
    for (int i = 0; i < 4; ++i)
      for (int at = 0; at < fd.NAT; ++at)
        for (int l = 0; l < 64; ++l) {
          int q = 16 * qt + rowof(i, l >> 4), al = 16 * at + (l & 15);
          if (q >= s.nqv || al >= nP) continue;
          for (int b = 0; b < dim; ++b)
            f.vol_dVT[(((qt * 4 + i) * dim + b) * fd.NAT + at) * 64 + l] = t.dV[(q * nP + al) * dim + b];
          f.vol_VT[((qt * 4 + i) * fd.NAT + at) * 64 + l] = t.V[q * nP + al];
        }
  // facets
  f.fac_Tr.assign((dim + 1) * fd.NQFT * fd.NPK * 64, 0.0);
  f.fac_TrT.assign((dim + 1) * fd.NQFT * 4 * fd.NAT * 64, 0.0);
  f.fac_K.assign((dim + 1) * fd.NFJT * fd.NPK * 64, 0.0);
  f.fac_KT.assign((dim + 1) * fd.NAT * fd.NFK * 64, 0.0);
  for (int fc = 0; fc <= dim; ++fc) {
    for (int qt = 0; qt < fd.NQFT; ++qt) {
      for (int kk = 0; kk < fd.NPK; ++kk)
        for (int l = 0; l < 64; ++l) {
          int q = 16 * qt + (l & 15), al = 4 * kk + (l >> 4);
          if (q >= s.nqf || al >= nP) continue;
          f.fac_Tr[((fc * fd.NQFT + qt) * fd.NPK + kk) * 64 + l] = t.Tr[(fc * s.nqf + q) * nP + al];
        }
      for (int i = 0; i < 4; ++i)
        for (int at = 0; at < fd.NAT; ++at)
          for (int l = 0; l < 64; ++l) {
            int q = 16 * qt + rowof(i, l >> 4), al = 16 * at + (l & 15);
            if (q >= s.nqf || al >= nP) continue;
            f.fac_TrT[(((fc * fd.NQFT + qt) * 4 + i) * fd.NAT + at) * 64 + l] = t.Tr[(fc * s.nqf + q) * nP + al];
          }
    }
    for (int jt = 0; jt < fd.NFJT; ++jt)
      for (int kk = 0; kk < fd.NPK; ++kk)
        for (int l = 0; l < 64; ++l) {
          int j = 16 * jt + (l & 15), al = 4 * kk + (l >> 4);
          if (j >= nf || al >= nP) continue;
          f.fac_K[((fc * fd.NFJT + jt) * fd.NPK + kk) * 64 + l] = t.Kf[(fc * nf + j) * nP + al];
        }
    for (int at = 0; at < fd.NAT; ++at)
      for (int jk = 0; jk < fd.NFK; ++jk)
        for (int l = 0; l < 64; ++l) {
          int j = 16 * (jk / 4) + rowof(jk % 4, l >> 4), al = 16 * at + (l & 15);
          if (j >= nf || al >= nP) continue;
          f.fac_KT[((fc * fd.NAT + at) * fd.NFK + jk) * 64 + l] = t.Kf[(fc * nf + j) * nP + al];
        }
  }
  // u.n at the facet points from the facet DoFs by an f64 MFMA (every
  // precision form): the f64 MFMA puts output row 4i + g in register i of
  // lane group g, so row 4i + g holds this row map's point rowof(i, g)
  f.psi_n.assign(fd.NQFT * fd.NFK * 64, 0.0);
  for (int qt = 0; qt < fd.NQFT; ++qt)
    for (int jk = 0; jk < fd.NFK; ++jk)
      for (int l = 0; l < 64; ++l) {
        const int m = l & 15;
        const int q = 16 * qt + rowof(m / 4, m % 4), j = 4 * jk + (l >> 4);
        if (q >= s.nqf || j >= nf) continue;
        f.psi_n[(qt * fd.NFK + jk) * 64 + l] = t.Psi[q * nf + j];
      }
  f.fac_Psi.assign(fd.NQFT * fd.NFK * 64, 0.0);
  f.fac_PsiT.assign(fd.NQFT * 4 * fd.NFJT * 64, 0.0);
  for (int qt = 0; qt < fd.NQFT; ++qt) {
    for (int jk = 0; jk < fd.NFK; ++jk)
      for (int l = 0; l < 64; ++l) {
        int q = 16 * qt + (l & 15), j = 16 * (jk / 4) + rowof(jk % 4, l >> 4);
        if (q >= s.nqf || j >= nf) continue;
        f.fac_Psi[(qt * fd.NFK + jk) * 64 + l] = t.Psi[q * nf + j];
      }
    for (int i = 0; i < 4; ++i)
      for (int jt = 0; jt < fd.NFJT; ++jt)
        for (int l = 0; l < 64; ++l) {
          int q = 16 * qt + rowof(i, l >> 4), j = 16 * jt + (l & 15);
          if (q >= s.nqf || j >= nf) continue;
          f.fac_PsiT[((qt * 4 + i) * fd.NFJT + jt) * 64 + l] = t.wf[q] * t.Psi[q * nf + j];
        }
  }
  // dual (element kernel): rows j, k over (a, alpha tile, reg)
  f.dual.assign(fd.NJT * dim * fd.NAT * 4 * 64, 0.0);
  for (int jt = 0; jt < fd.NJT; ++jt)
    for (int a = 0; a < dim; ++a)
      for (int at = 0; at < fd.NAT; ++at)
        for (int i = 0; i < 4; ++i)
          for (int l = 0; l < 64; ++l) {
            int j = 16 * jt + (l & 15), al = 16 * at + rowof(i, l >> 4);
            if (j >= n || al >= nP) continue;
            f.dual[((((jt * dim + a) * fd.NAT + at) * 4) + i) * 64 + l] = Dinv(a, al, j);
          }
}

// ------------------------------------------------------------ mesh
bool build_mesh(int dim, int64_t E, const int64_t* elem_vid, const double* elem_xyz,
                MeshData& m, std::string& err) {
  const int dp1 = dim + 1;
  m.dim = dim;
  m.E = E;
  m.vid.resize(E * dp1);
  m.xyz.resize(E * dp1 * dim);
  m.geo.assign(E * GEO_STRIDE, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    int ord[4] = {0, 1, 2, 3};
    std::sort(ord, ord + dp1, [&](int a, int b) { return elem_vid[e * dp1 + a] < elem_vid[e * dp1 + b]; });
    for (int i = 0; i < dp1; ++i) {
      m.vid[e * dp1 + i] = elem_vid[e * dp1 + ord[i]];
      for (int a = 0; a < dim; ++a) m.xyz[(e * dp1 + i) * dim + a] = elem_xyz[(e * dp1 + ord[i]) * dim + a];
      if (i > 0 && m.vid[e * dp1 + i] == m.vid[e * dp1 + i - 1]) {
        err = "element " + std::to_string(e) + " has a repeated vertex";
        return false;
      }
    }
    double* g = &m.geo[e * GEO_STRIDE];
    const double* x = &m.xyz[e * dp1 * dim];
    for (int r = 0; r < dim; ++r)
      for (int c = 0; c < dim; ++c) g[r * dim + c] = x[(c + 1) * dim + r] - x[r];
    double det;
    if (dim == 2) det = g[0] * g[3] - g[1] * g[2];
    else det = g[0] * (g[4] * g[8] - g[5] * g[7]) - g[1] * (g[3] * g[8] - g[5] * g[6]) + g[2] * (g[3] * g[7] - g[4] * g[6]);
    if (!(det != 0.0) || !std::isfinite(det)) {
      err = "element " + std::to_string(e) + " is degenerate (det J = 0)";
      return false;
    }
    g[GEO_DET] = det;
    for (int i = 0; i < dp1; ++i) {
      int lv[3], c = 0;
      for (int v = 0; v < dp1; ++v) if (v != i) lv[c++] = v;
      double N[3];
      double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) t1[a] = x[lv[1] * dim + a] - x[lv[0] * dim + a];
      if (dim == 2) { N[0] = t1[1]; N[1] = -t1[0]; }
      else {
        for (int a = 0; a < 3; ++a) t2[a] = x[lv[2] * 3 + a] - x[lv[0] * 3 + a];
        N[0] = t1[1] * t2[2] - t1[2] * t2[1];
        N[1] = t1[2] * t2[0] - t1[0] * t2[2];
        N[2] = t1[0] * t2[1] - t1[1] * t2[0];
      }
      double nn = 0;
      for (int a = 0; a < dim; ++a) nn += N[a] * N[a];
      nn = std::sqrt(nn);
      double sigma = ((i % 2) ? -1.0 : 1.0) * (det > 0 ? 1.0 : -1.0);
      g[GEO_NFN + i] = nn;
      for (int a = 0; a < dim; ++a) g[GEO_NRM + i * dim + a] = sigma * N[a] / nn;
    }
  }
  // facets: sort (key, element, local)
  struct Key { int64_t v[3]; int64_t e; int i; };
  std::vector<Key> keys(E * dp1);
  for (int64_t e = 0; e < E; ++e)
    for (int i = 0; i < dp1; ++i) {
      Key& k = keys[e * dp1 + i];
      int c = 0;
      for (int v = 0; v < dp1; ++v) if (v != i) k.v[c++] = m.vid[e * dp1 + v];
      for (; c < 3; ++c) k.v[c] = -1;
      k.e = e; k.i = i;
    }
  std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
    for (int c = 0; c < 3; ++c) if (a.v[c] != b.v[c]) return a.v[c] < b.v[c];
    if (a.e != b.e) return a.e < b.e;
    return a.i < b.i;
  });
  m.fid.assign(E * dp1, -1);
  m.nbr.assign(E * dp1, -1);
  m.nbr_face.assign(E * dp1, -1);
  m.facet_elem.clear();
  m.facet_local.clear();
  int64_t F = 0, W = 0;
  size_t p = 0;
  while (p < keys.size()) {
    size_t q = p + 1;
    while (q < keys.size() && keys[q].v[0] == keys[p].v[0] && keys[q].v[1] == keys[p].v[1] && keys[q].v[2] == keys[p].v[2]) ++q;
    size_t cnt = q - p;
    if (cnt > 2) { err = "a facet is shared by more than two elements"; return false; }
    if (cnt == 1) { ++W; }
    else {
      const Key& a = keys[p]; const Key& b = keys[p + 1];
      if (a.e == b.e) { err = "element " + std::to_string(a.e) + " is its own neighbour (a periodic direction needs at least 3 cells)"; return false; }
      if (F > INT32_MAX - 1) { err = "too many facets"; return false; }
      m.fid[a.e * dp1 + a.i] = (int32_t)F;
      m.fid[b.e * dp1 + b.i] = (int32_t)F;
      m.nbr[a.e * dp1 + a.i] = (int32_t)b.e;
      m.nbr[b.e * dp1 + b.i] = (int32_t)a.e;
      m.nbr_face[a.e * dp1 + a.i] = (int8_t)b.i;
      m.nbr_face[b.e * dp1 + b.i] = (int8_t)a.i;
      m.facet_elem.push_back((int32_t)a.e);
      m.facet_elem.push_back((int32_t)b.e);
      m.facet_local.push_back((int8_t)a.i);
      m.facet_local.push_back((int8_t)b.i);
      ++F;
    }
    p = q;
  }
  m.F = F;
  m.W = W;
  return true;
}

void make_batches(const MeshData& m, Batches& b) {
  const int dp1 = m.dim + 1;
  std::vector<int32_t> sig(m.E);
  for (int64_t e = 0; e < m.E; ++e) {
    int32_t s = 0;
    for (int f = 0; f < dp1; ++f) {
      int code = m.nbr[e * dp1 + f] < 0 ? 0xF : m.nbr_face[e * dp1 + f];
      s |= code << (4 * f);
    }
    sig[e] = s;
  }
  std::vector<int64_t> order(m.E);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t c) { return sig[a] < sig[c]; });
  struct B { int32_t first; int32_t sig; std::array<int32_t, 16> el; };
  std::vector<B> bs;
  size_t p = 0;
  while (p < order.size()) {
    B cur;
    cur.sig = sig[order[p]];
    cur.el.fill(-1);
    int c = 0;
    while (p < order.size() && c < 16 && sig[order[p]] == cur.sig) cur.el[c++] = (int32_t)order[p++];
    cur.first = cur.el[0];
    bs.push_back(cur);
  }
  // spatial order: by the first element of each batch
  std::stable_sort(bs.begin(), bs.end(), [](const B& a, const B& c) { return a.first < c.first; });
  b.nb = (int64_t)bs.size();
  b.elem.resize(b.nb * 16);
  b.sig.resize(b.nb);
  for (int64_t i = 0; i < b.nb; ++i) {
    b.sig[i] = bs[i].sig;
    for (int c = 0; c < 16; ++c) b.elem[i * 16 + c] = bs[i].el[c];
  }
}

}  // namespace hopu
