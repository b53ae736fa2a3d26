// Device kernels of the implicit Stokes step (paper section 2.3, eq.
// (MCS_step1), static condensation and the element-wise BDDC).
//
// Set-up, one workgroup per element (persistent over elements):
//   G   [ng][nsf]  the element's constraint rows against the full trace-free
//                  P^{k+1} stress basis E_a p_alpha (orthonormal, so the
//                  stress mass block is D = -|det J|/(2 nu) I):
//                  rows gamma (c, beta), nt multipliers (facet, tangent, top
//                  mode), velocity DoFs, u^ unknowns;
//   K   = -(2 nu/|det J|) G G^t  (LDS-tiled Gram);
//   -K11 = L L^t (Cholesky), W^t = K21 L^-t, S_T = A_T - K22 - W^t W with
//   A_T = [M_T/dt, 0; 0, 0];
//   S_T = L_S L_S^t, X = L_S^-1, S_T^-1 = X^t X.
// Wall unknowns (u^ and the multipliers on wall facets) have zero rows; their
// diagonals are set to one so that every factorisation stays defined.
//
// The set-up stores the upper triangles of S_T and S_T^-1, packed by rows
// (S_T^-1 optionally in FP32).  PCG, one workgroup per element: y_T = A_T x_T
// with A_T = S_T or S_T^-1 read once from HBM, facet unknowns written per
// side and summed per facet in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "launch_events.hpp"
#include "stokes.hpp"

namespace hopu {

namespace {

constexpr int ST_THREADS = 256;
constexpr int TILE = 64;
constexpr int KCH = 16;

// C[i][j] (= or +=) scale * sum_k A[i][k] A[j][k] for i, j < m (full
// symmetric result); A row stride lda, C row stride ldc; whole workgroup.
__device__ void block_gram(const double* A, int lda, int m, int kd, double* C, int ldc, double scale,
                           bool accumulate, double* As, double* Bs) {
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int nt = (m + TILE - 1) / TILE;
  for (int ti = 0; ti < nt; ++ti)
    for (int tj = 0; tj <= ti; ++tj) {
      double acc[4][4];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int k0 = 0; k0 < kd; k0 += KCH) {
        for (int v = t; v < TILE * KCH; v += ST_THREADS) {
          const int r = v / KCH, c = v % KCH;
          const int ia = ti * TILE + r, ib = tj * TILE + r, kc = k0 + c;
          As[r * (KCH + 1) + c] = (ia < m && kc < kd) ? A[(size_t)ia * lda + kc] : 0.0;
          Bs[r * (KCH + 1) + c] = (ib < m && kc < kd) ? A[(size_t)ib * lda + kc] : 0.0;
        }
        __syncthreads();
        for (int c = 0; c < KCH; ++c) {
          double av[4], bv[4];
          for (int a = 0; a < 4; ++a) av[a] = As[(ty * 4 + a) * (KCH + 1) + c];
          for (int b = 0; b < 4; ++b) bv[b] = Bs[(tx * 4 + b) * (KCH + 1) + c];
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
      }
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const int i = ti * TILE + ty * 4 + a, j = tj * TILE + tx * 4 + b;
          if (i >= m || j >= m) continue;
          const double v = scale * acc[a][b];
          if (accumulate) {
            C[(size_t)i * ldc + j] += v;
            if (ti != tj) C[(size_t)j * ldc + i] += v;
          } else {
            C[(size_t)i * ldc + j] = v;
            if (ti != tj) C[(size_t)j * ldc + i] = v;
          }
        }
    }
  __syncthreads();
}

// In-place lower Cholesky of the n x n matrix at A (row stride lda); the
// strict upper triangle is left as it was.  Raises *bad on a pivot <= 0.
__device__ void block_cholesky(double* A, int lda, int n, int* bad) {
  const int t = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    __shared__ double piv;
    if (t == 0) {
      double a = A[(size_t)j * lda + j];
      if (!(a > 0.0)) {
        atomicAdd(bad, 1);
        a = 1.0;
      }
      piv = sqrt(a);
      A[(size_t)j * lda + j] = piv;
    }
    __syncthreads();
    const double ip = 1.0 / piv;
    for (int i = j + 1 + t; i < n; i += ST_THREADS) A[(size_t)i * lda + j] *= ip;
    __syncthreads();
    // trailing update of the lower triangle: rows i > j, columns j < c <= i
    const int r = n - j - 1;
    const int64_t tot = (int64_t)r * (r + 1) / 2;
    for (int64_t v = t; v < tot; v += ST_THREADS) {
      // v -> (ii, cc) with 0 <= cc <= ii < r
      int ii = (int)((sqrt(8.0 * (double)v + 1.0) - 1.0) * 0.5);
      while ((int64_t)(ii + 1) * (ii + 2) / 2 <= v) ++ii;
      while ((int64_t)ii * (ii + 1) / 2 > v) --ii;
      const int cc = (int)(v - (int64_t)ii * (ii + 1) / 2);
      const int i = j + 1 + ii, c = j + 1 + cc;
      A[(size_t)i * lda + c] -= A[(size_t)i * lda + j] * A[(size_t)c * lda + j];
    }
    __syncthreads();
  }
}

// Upper triangle of the symmetric n x n matrix A (row stride n), packed by
// rows: row i holds A[i][i..n-1] at offset i n - i (i - 1)/2.
template <typename OT>
__device__ void pack_upper(const double* A, int n, OT* out) {
  for (int64_t v = threadIdx.x; v < (int64_t)n * n; v += ST_THREADS) {
    const int i = (int)(v / n), j = (int)(v % n);
    if (j >= i) out[(int64_t)i * n - (int64_t)i * (i - 1) / 2 + (j - i)] = (OT)A[v];
  }
  __syncthreads();
}

__device__ inline int64_t gidx(const StokesDims& sd, const StokesDev& dv, int64_t e, int t, int* fside, int* vslot) {
  const int dp1 = sd.dim + 1;
  const int nfl = dp1 * sd.nf;
  if (t < nfl) {
    const int f = t / sd.nf, j = t % sd.nf;
    const int32_t F = dv.fid[e * dp1 + f];
    *fside = f;
    *vslot = j;
    return F >= 0 ? (int64_t)F * sd.nf + j : -1;
  }
  if (t < sd.n) {
    *fside = -1;
    return dv.F * sd.nf + e * sd.nint + (t - nfl);
  }
  const int th = t - sd.n;
  const int per = (sd.dim - 1) * sd.nf;
  const int f = th / per, rem = th % per;
  const int c = rem / sd.nf, j = rem % sd.nf;
  const int32_t F = dv.fid[e * dp1 + f];
  *fside = f;
  *vslot = sd.nf + c * sd.nf + j;
  return F >= 0 ? dv.n_dof + ((int64_t)F * (sd.dim - 1) + c) * sd.nf + j : -1;
}

}  // namespace

__global__ void __launch_bounds__(ST_THREADS)
    k_stokes_setup(StokesDims sd, StokesDev dv, double nu, double dt, double* __restrict__ ST,
                   double* __restrict__ STinv, float* __restrict__ STinv32, double* __restrict__ scratch,
                   int* bad) {
  __shared__ double As[TILE * (KCH + 1)], Bs[TILE * (KCH + 1)];
  __shared__ double H[8 * 9];   // J^-1 E_a^T J
  __shared__ double Gm[9];      // J^T J
  __shared__ double geo[STG];
  const int d = sd.dim, t = threadIdx.x;
  const int ng = sd.ng, nsf = sd.nsf, nx = sd.nx, n1 = sd.n1;
  double* G = scratch + (size_t)blockIdx.x * ((size_t)ng * nsf + (size_t)ng * ng);
  double* K = G + (size_t)ng * nsf;
  for (int64_t e = blockIdx.x; e < dv.E; e += gridDim.x) {
    if (t < STG) geo[t] = dv.sgeo[e * STG + t];
    __syncthreads();
    const double det = geo[18], adet = fabs(det), sgn = det > 0 ? 1.0 : -1.0;
    if (t < sd.nE * 9) {
      const int a = t / 9, r = (t % 9) / 3, s = t % 3;
      double v = 0.0;
      if (r < d && s < d)
        for (int p = 0; p < d; ++p)
          for (int q = 0; q < d; ++q)  // (J^-1)_{rp} (E_a)_{qp} J_{qs}
            v += geo[9 + r * 3 + p] * dv.Ea[(a * d + q) * d + p] * geo[q * 3 + s];
      H[t] = v;
    }
    if (t < 9) {
      const int r = t / 3, s = t % 3;
      double v = 0.0;
      for (int q = 0; q < d; ++q) v += geo[q * 3 + r] * geo[q * 3 + s];
      Gm[t] = v;
    }
    __syncthreads();
    // ---- G
    const int ngam = sd.nG * sd.nPk;
    const double pint = pow(adet, (double)(d - 1) / (double)d);
    for (int64_t v = t; v < (int64_t)ng * nsf; v += ST_THREADS) {
      const int row = (int)(v / nsf), col = (int)(v % nsf);
      const int a = col / sd.nP1, al = col % sd.nP1;
      const double* Ea = dv.Ea + a * d * d;
      double g = 0.0;
      if (row < ngam) {
        const int c = row / sd.nPk, be = row % sd.nPk;
        double ge = 0.0;
        for (int q = 0; q < d * d; ++q) ge += dv.Gc[c * d * d + q] * Ea[q];
        g = -adet * ge * dv.MpG[be * sd.nP1 + al];
      } else if (row < n1) {
        const int rr = row - ngam;
        const int per = (d - 1) * sd.ntop;
        const int f = rr / per, c = (rr % per) / sd.ntop, m = rr % sd.ntop;
        const double* fr = geo + 20 + 11 * f;
        if (fr[10] > 0.5) {
          double ent = 0.0;  // n . E_a t_c
          for (int p = 0; p < d; ++p)
            for (int q = 0; q < d; ++q) ent += fr[p] * Ea[p * d + q] * fr[3 + 3 * c + q];
          g = adet * ent * dv.Phi[((size_t)f * sd.nP1 + al) * sd.nft + sd.nf + m];
        }
      } else if (row < n1 + sd.n) {
        const int i = row - n1;
        const double* tv = dv.TV + ((size_t)al * sd.n + i) * d * d;
        double vol = 0.0;
        for (int r = 0; r < d; ++r)
          for (int s = 0; s < d; ++s) vol += H[a * 9 + r * 3 + s] * tv[r * d + s];
        const int nfl = (d + 1) * sd.nf;
        if (i < nfl) {
          const int f = i / sd.nf, j = i % sd.nf;
          const double* fr = geo + 20 + 11 * f;
          const double sf = ((f % 2) ? -1.0 : 1.0) * sgn;  // outward sign of the facet's n_F
          double enn = 0.0;
          for (int p = 0; p < d; ++p)
            for (int q = 0; q < d; ++q) enn += fr[p] * Ea[p * d + q] * fr[q];
          g = -fr[9] * sgn * vol + sf * fr[9] * enn * dv.Phi[((size_t)f * sd.nP1 + al) * sd.nft + j];
        } else {
          g = -pint * sgn * vol;
        }
      } else {
        const int th = row - n1 - sd.n;
        const int per = (d - 1) * sd.nf;
        const int f = th / per, c = (th % per) / sd.nf, j = th % sd.nf;
        const double* fr = geo + 20 + 11 * f;
        if (fr[10] > 0.5) {
          double etn = 0.0;  // t_c . E_a n_out
          for (int p = 0; p < d; ++p)
            for (int q = 0; q < d; ++q) etn += fr[3 + 3 * c + p] * Ea[p * d + q] * fr[q];
          g = fr[9] * etn * dv.Phi[((size_t)f * sd.nP1 + al) * sd.nft + j];
        }
      }
      G[v] = g;
    }
    __syncthreads();
    // ---- K = -(2 nu / |det J|) G G^t
    block_gram(G, nsf, ng, nsf, K, ng, -2.0 * nu / adet, false, As, Bs);
    // wall multipliers and wall u^ unknowns: unit diagonal (their rows are zero)
    for (int row = t; row < ng; row += ST_THREADS) {
      bool wall = false;
      if (row >= ngam && row < n1) {
        const int f = (row - ngam) / ((d - 1) * sd.ntop);
        wall = geo[20 + 11 * f + 10] < 0.5;
      } else if (row >= n1 + sd.n) {
        const int f = (row - n1 - sd.n) / ((d - 1) * sd.nf);
        wall = geo[20 + 11 * f + 10] < 0.5;
      }
      if (wall) K[(size_t)row * ng + row] = row < n1 ? -1.0 : 0.0;
    }
    __syncthreads();
    // ---- -K11 = L L^t
    for (int64_t v = t; v < (int64_t)n1 * n1; v += ST_THREADS) {
      const int i = (int)(v / n1), j = (int)(v % n1);
      K[(size_t)i * ng + j] = -K[(size_t)i * ng + j];
    }
    __syncthreads();
    block_cholesky(K, ng, n1, bad);
    // ---- W^t = K21 L^-t (rows of K21 by forward substitution), in place
    for (int r = t; r < nx; r += ST_THREADS) {
      double* w = K + (size_t)(n1 + r) * ng;
      for (int j = 0; j < n1; ++j) {
        double v = w[j];
        for (int m = 0; m < j; ++m) v -= K[(size_t)j * ng + m] * w[m];
        w[j] = v / K[(size_t)j * ng + j];
      }
    }
    __syncthreads();
    // ---- K22 += W^t W; S_T = A_T - K22 (formed in full, then packed into ST)
    double* K22 = K + (size_t)n1 * ng + n1;
    block_gram(K + (size_t)n1 * ng, ng, nx, n1, K22, ng, 1.0, true, As, Bs);
    // S_T in full (row stride nx) in G's storage, which is free once K is formed
    double* S = G;
    for (int64_t v = t; v < (int64_t)nx * nx; v += ST_THREADS) {
      const int i = (int)(v / nx), j = (int)(v % nx);
      double s = -K22[(size_t)i * ng + j];
      if (i < sd.n && j < sd.n) {
        const int nfl = (d + 1) * sd.nf;
        const double si = i < nfl ? geo[20 + 11 * (i / sd.nf) + 9] : pint;
        const double sj = j < nfl ? geo[20 + 11 * (j / sd.nf) + 9] : pint;
        const double* mr = dv.Mref + ((size_t)i * sd.n + j) * d * d;
        double m = 0.0;
        for (int r = 0; r < d; ++r)
          for (int q = 0; q < d; ++q) m += Gm[r * 3 + q] * mr[r * d + q];
        s += si * sj / adet * m / dt;
      }
      // velocity DoFs on wall facets and wall u^: unit rows and columns
      bool wi = false, wj = false;
      {
        const int nfl = (d + 1) * sd.nf;
        if (i < nfl) wi = geo[20 + 11 * (i / sd.nf) + 10] < 0.5;
        else if (i >= sd.n) wi = geo[20 + 11 * ((i - sd.n) / ((d - 1) * sd.nf)) + 10] < 0.5;
        if (j < nfl) wj = geo[20 + 11 * (j / sd.nf) + 10] < 0.5;
        else if (j >= sd.n) wj = geo[20 + 11 * ((j - sd.n) / ((d - 1) * sd.nf)) + 10] < 0.5;
      }
      if (wi || wj) s = (i == j) ? 1.0 : 0.0;
      S[v] = s;
    }
    __syncthreads();
    pack_upper(S, nx, ST + (size_t)e * stokes_packed_stride(nx));
    // ---- S_T^-1: L_S L_S^t = S_T in place, X = L_S^-1 stored transposed in
    // K's storage (row stride nx), S_T^-1 = X^t X into G's storage, packed
    block_cholesky(S, nx, nx, bad);
    double* XT = K;
    for (int i = t; i < nx; i += ST_THREADS) {
      double* xt = XT + (size_t)i * nx;  // row i: X[m][i] for m = 0..nx-1
      for (int m = 0; m < i; ++m) xt[m] = 0.0;
      xt[i] = 1.0 / S[(size_t)i * nx + i];
      for (int m = i + 1; m < nx; ++m) {
        double v = 0.0;
        for (int p = i; p < m; ++p) v += S[(size_t)m * nx + p] * xt[p];
        xt[m] = -v / S[(size_t)m * nx + m];
      }
    }
    __syncthreads();
    block_gram(XT, nx, nx, nx, S, nx, 1.0, false, As, Bs);
    if (STinv32) pack_upper(S, nx, STinv32 + (size_t)e * stokes_packed_stride(nx));
    else pack_upper(S, nx, STinv + (size_t)e * stokes_packed_stride(nx));
  }
}

// y_T = A_T (w x_T) with w = 1/2 on facet unknowns for the preconditioner
// (R^t) and the same weight on the way out (R).  A_T is read once, as its
// packed upper triangle.  A quarter-wave (16 lanes) owns one row: wave w
// takes the row groups 4g .. 4g+3 with g = w, w + 4, ...; a row's lanes load
// A[i][j], j >= i, in chunks of 16 (all chunks of the row in flight at once)
// and give both its dot product with x (row i of y, a 16-lane reduction)
// and the symmetric part A[i][j] x_i for the rows j > i, added to the
// quarter's own partial y in LDS.  Every sum has a fixed order, so results
// are bitwise reproducible.
// CH = ceil(nx / 16) chunks per row (nx <= 16 CH).  The first row group's
// loads are issued before the gather of x, each later group's at the end of
// the previous one (a second register set for a deeper prefetch halves the
// resident waves and measured slower).
template <int CH, typename MT>
__global__ void __launch_bounds__(ST_THREADS)
    k_stokes_gemv(StokesDims sd, StokesDev dv, const MT* __restrict__ A, int inv, const double* __restrict__ x,
                  double* __restrict__ y, double* __restrict__ slot) {
  extern __shared__ double lds[];
  const int nx = sd.nx;
  double* xs = lds;            // [nx]
  double* yr = lds + nx;       // [nx]  row dots
  double* yp = lds + 2 * nx;   // [16][nx] partials of the symmetric part, per quarter-wave
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  const int q = lane / 16, s16 = lane % 16;
  const int64_t e = blockIdx.x;
  const double wf = inv ? 0.5 : 1.0;
  const MT* Ae = A + (size_t)e * stokes_packed_stride(nx);
  // the row group's loads land in registers of the stored type; FP32
  // matrices keep two groups in flight per wave (same register budget as
  // one FP64 group)
  auto load_group = [&](int g, MT* v) {
    const int i = 4 * g + q;
    const MT* row = Ae + ((int64_t)i * nx - (int64_t)i * (i - 1) / 2) - i;  // row[j] = A[i][j]
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = i + s16 + 16 * c;
      v[c] = (i < nx && j < nx) ? __builtin_nontemporal_load(row + j) : (MT)0;
    }
  };
  double* ypq = yp + (size_t)(4 * w + q) * nx;
  auto use_group = [&](int g, const MT* v) {
    const int i = 4 * g + q;
    double dot = 0.0;
    if (i < nx) {
      const double xi = xs[i];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = i + s16 + 16 * c;
        if (j < nx) {
          dot += (double)v[c] * xs[j];
          if (j > i) ypq[j] += (double)v[c] * xi;
        }
      }
    }
    for (int off = 8; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 16);
    if (s16 == 0 && i < nx) yr[i] = dot;
  };
  auto gather = [&]() {
    for (int i = t; i < nx; i += ST_THREADS) {
      int fs = -1, vs = 0;
      const int64_t g = gidx(sd, dv, e, i, &fs, &vs);
      xs[i] = g >= 0 ? (fs >= 0 ? wf : 1.0) * x[g] : 0.0;
    }
    for (int k = t; k < 16 * nx; k += ST_THREADS) yp[k] = 0.0;
    __syncthreads();
  };
  if constexpr (sizeof(MT) == 4) {
    MT va[CH], vb[CH];
    load_group(w, va);
    if (4 * (w + 4) < nx) load_group(w + 4, vb);
    gather();
    for (int g = w; 4 * g < nx; g += 8) {
      use_group(g, va);
      if (4 * (g + 8) < nx) load_group(g + 8, va);
      if (4 * (g + 4) < nx) {
        use_group(g + 4, vb);
        if (4 * (g + 12) < nx) load_group(g + 12, vb);
      }
    }
  } else {
    MT v[CH];
    load_group(w, v);
    gather();
    for (int g = w; 4 * g < nx; g += 4) {
      use_group(g, v);
      if (4 * (g + 4) < nx) load_group(g + 4, v);
    }
  }
  __syncthreads();
  for (int i = t; i < nx; i += ST_THREADS) {
    double sym = 0.0;
    for (int p = 0; p < 16; ++p) sym += yp[(size_t)p * nx + i];
    const double val = yr[i] + sym;
    int fs = -1, vs = 0;
    const int64_t g = gidx(sd, dv, e, i, &fs, &vs);
    if (g >= 0) {
      if (fs < 0) y[g] = val;
      else slot[((size_t)e * (sd.dim + 1) + fs) * sd.nsd + vs] = wf * val;
    }
  }
}

__global__ void k_stokes_facets(StokesDims sd, StokesDev dv, const double* __restrict__ slot, double* __restrict__ y) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= dv.F * sd.nsd) return;
  const int64_t F = v / sd.nsd;
  const int c = (int)(v % sd.nsd);
  const int dp1 = sd.dim + 1;
  const int32_t T0 = dv.facet_elem[2 * F], T1 = dv.facet_elem[2 * F + 1];
  const int f0 = dv.facet_local[2 * F], f1 = dv.facet_local[2 * F + 1];
  const double s = slot[((size_t)T0 * dp1 + f0) * sd.nsd + c] + slot[((size_t)T1 * dp1 + f1) * sd.nsd + c];
  if (c < sd.nf) y[F * sd.nf + c] = s;
  else {
    const int cc = (c - sd.nf) / sd.nf, j = (c - sd.nf) % sd.nf;
    y[dv.n_dof + (F * (sd.dim - 1) + cc) * sd.nf + j] = s;
  }
}

constexpr int NPART_ST = 1024;

__global__ void __launch_bounds__(256) k_stokes_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                    int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_stokes_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ void k_stokes_xpby(double* __restrict__ p, const double* __restrict__ z, double b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + b * p[i];
}

__global__ void k_stokes_rhs(double* __restrict__ y, const double* __restrict__ Mu, const double* __restrict__ r,
                             double dt, int64_t n_dof, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = i < n_dof ? Mu[i] / dt - (r ? r[i] : 0.0) : 0.0;
}

int stokes_setup_blocks(const StokesDims&) { return 2048; }

size_t stokes_setup_scratch(const StokesDims& sd) {
  return (size_t)stokes_setup_blocks(sd) * ((size_t)sd.ng * sd.nsf + (size_t)sd.ng * sd.ng);
}

void launch_stokes_setup(hipStream_t s, const StokesDims& sd, const StokesDev& dv, double nu, double dt, double* ST,
                         double* STinv, float* STinv32, double* scratch, int* bad) {
  const int nb = (int)std::min<int64_t>(stokes_setup_blocks(sd), dv.E);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_stokes_setup, dim3(nb), dim3(ST_THREADS), 0, s, sd, dv, nu, dt, ST, STinv, STinv32, scratch,
                     bad);
}

template <typename MT>
static void gemv_dispatch(hipStream_t s, const StokesDims& sd, const StokesDev& dv, const MT* A, int inv,
                          const double* x, double* y, double* slot) {
  const size_t lds = (size_t)18 * sd.nx * sizeof(double);
  const int ch = (sd.nx + 15) / 16;
  const dim3 grid((unsigned)dv.E), blk(ST_THREADS);
  if (ch <= 1) HOPU_LAUNCH((k_stokes_gemv<1, MT>), grid, blk, lds, s, sd, dv, A, inv, x, y, slot);
  else if (ch <= 2) HOPU_LAUNCH((k_stokes_gemv<2, MT>), grid, blk, lds, s, sd, dv, A, inv, x, y, slot);
  else if (ch <= 3) HOPU_LAUNCH((k_stokes_gemv<3, MT>), grid, blk, lds, s, sd, dv, A, inv, x, y, slot);
  else if (ch <= 5) HOPU_LAUNCH((k_stokes_gemv<5, MT>), grid, blk, lds, s, sd, dv, A, inv, x, y, slot);
  else if (ch <= 9) HOPU_LAUNCH((k_stokes_gemv<9, MT>), grid, blk, lds, s, sd, dv, A, inv, x, y, slot);
  else HOPU_LAUNCH((k_stokes_gemv<16, MT>), grid, blk, lds, s, sd, dv, A, inv, x, y, slot);
}

void launch_stokes_gemv(hipStream_t s, const StokesDims& sd, const StokesDev& dv, const double* A, const float* A32,
                        int inv, const double* x, double* y, double* slot) {
  if (dv.E > 0) {
    if (A32) gemv_dispatch(s, sd, dv, A32, inv, x, y, slot);
    else gemv_dispatch(s, sd, dv, A, inv, x, y, slot);
  }
  const int64_t nv = dv.F * sd.nsd;
  if (nv > 0) hipLaunchKernelGGL(k_stokes_facets, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, sd, dv, slot, y);
}

int launch_stokes_dot(hipStream_t s, const double* a, const double* b, int64_t n, double* part) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(NPART_ST, (n + 255) / 256));
  hipLaunchKernelGGL(k_stokes_dot, dim3(nb), dim3(256), 0, s, a, b, n, part);
  return nb;
}

void launch_stokes_axpy(hipStream_t s, double* y, const double* x, double a, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_stokes_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, x, a, n);
}

void launch_stokes_xpby(hipStream_t s, double* p, const double* z, double b, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_stokes_xpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, z, b, n);
}

void launch_stokes_rhs(hipStream_t s, double* y, const double* Mu, const double* r, double dt, int64_t n_dof,
                       int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_stokes_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, Mu, r, dt, n_dof, n);
}

}  // namespace hopu
