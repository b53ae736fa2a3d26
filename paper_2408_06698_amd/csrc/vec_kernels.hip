// Vector kernels: deterministic two-stage dot products, PCG scalar updates,
// axpy-type updates, energy and divergence diagnostics.
#include <cstdint>

#include "vec.hpp"

namespace hopu {

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ part, const int* flag) {
  if (flag && *flag) return;
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += a[i] * b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Sum over a block of 256 threads of one value per thread in a fixed order:
// a butterfly inside each wave (lane 0's result is taken), then the four
// waves as (w0 + w1) + (w2 + w3).  Every block and every thread gets the
// same bits.  All threads of the block must call it; sh holds 4 doubles.
__device__ double block_sum_tree(double v, double* sh) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();  // sh may still be read from a previous call
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Sum of np partials: thread t adds part[t], part[t + 256], ... in order,
// then block_sum_tree.
__device__ double block_sum_fixed(const double* __restrict__ part, int np, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  return block_sum_tree(s, sh);
}

// Reduce partials in a fixed order and apply a PCG scalar operation.
__global__ __launch_bounds__(256) void k_scalar(const double* __restrict__ part, int np, double* sc, int* flag,
                                                int op, double arg, double* dst) {
  if (op != OP_SET_TOL && op != OP_STORE && op != OP_STORE_SQRT && flag && *flag) return;
  __shared__ double sh[4];
  const double v0 = block_sum_fixed(part, np, sh);
  if (threadIdx.x != 0) return;
  const double v = v0;
  switch (op) {
    case OP_SET_TOL:  // v = b.Pb
      sc[SC_TOL2] = arg * arg * v;
      sc[SC_BPB] = v;
      flag[0] = 0;
      flag[1] = 0;
      break;
    case OP_SET_RZ:
      sc[SC_RZ] = v;
      if (!(v > sc[SC_TOL2])) flag[0] = 1;
      sc[SC_RES] = sc[SC_BPB] > 0 ? sqrt(fmax(v, 0.0) / sc[SC_BPB]) : 0.0;
      break;
    case OP_STORE:
      *dst = v;
      break;
    case OP_STORE_SQRT:  // a norm from its squared partials
      *dst = sqrt(fmax(v, 0.0));
      break;
    default:
      break;
  }
}

// Vectors whose facet rows [0, nfl) are held unassembled as one contribution
// per facet side (fs[0][.] and fs[1][.]) and whose interior rows sit in place.
__device__ __forceinline__ double fs_row(const double* __restrict__ v, const double* __restrict__ fs, int64_t nfl,
                                         int64_t i) {
  return i < nfl ? fs[i] + fs[nfl + i] : v[i];
}

// Rows i and i + 1 (W = 2, 16-byte accesses) or row i (W = 1) of a vector
// whose facet rows [0, nfl) are unassembled.
template <int W> struct Rows;
template <> struct Rows<1> {
  double v[1];
  __device__ __forceinline__ void load(const double* __restrict__ a, int64_t i) { v[0] = a[i]; }
  __device__ __forceinline__ void load_fs(const double* __restrict__ a, const double* __restrict__ fs, int64_t nfl,
                                          int64_t i) {
    v[0] = fs_row(a, fs, nfl, i);
  }
  __device__ __forceinline__ void store(double* __restrict__ a, int64_t i) const { a[i] = v[0]; }
};
template <> struct Rows<2> {
  double v[2];
  __device__ __forceinline__ void load(const double* __restrict__ a, int64_t i) {
    const double2 t = *reinterpret_cast<const double2*>(a + i);
    v[0] = t.x;
    v[1] = t.y;
  }
  __device__ __forceinline__ void load_fs(const double* __restrict__ a, const double* __restrict__ fs, int64_t nfl,
                                          int64_t i) {
    if (i < nfl) {
      const double2 x = *reinterpret_cast<const double2*>(fs + i), y = *reinterpret_cast<const double2*>(fs + nfl + i);
      v[0] = x.x + y.x;
      v[1] = x.y + y.y;
    } else {
      load(a, i);
    }
  }
  __device__ __forceinline__ void store(double* __restrict__ a, int64_t i) const {
    *reinterpret_cast<double2*>(a + i) = make_double2(v[0], v[1]);
  }
};

// r -= alpha q (q unassembled).  With part: alpha = rz / (p.q), p.q the sum
// of the np partials of the operator launch before, reduced by every block
// in the same order (so every block holds the same alpha); block 0 records
// alpha (also in *arec if given) and the rz it divided.  With rr: each
// block's partial of r.r after the update (the inner product of an
// unpreconditioned CG).
template <int W>
__global__ __launch_bounds__(256) void k_rupdate(double* __restrict__ r, const double* __restrict__ q,
                                                 const double* __restrict__ fs, int64_t nfl, int64_t n, double* sc,
                                                 const int* flag, const double* __restrict__ part, int np,
                                                 double* __restrict__ rr, double* __restrict__ arec) {
  if (*flag) return;  // no launch of this kernel's iteration writes the flag
  __shared__ double sh[4];
  double al;
  if (part) {
    al = sc[SC_RZ] / block_sum_fixed(part, np, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[SC_ALPHA] = al;
      sc[SC_RZ_OLD] = sc[SC_RZ];
      if (arec) *arec = al;
    }
  } else {
    al = sc[SC_ALPHA];
  }
  double acc = 0.0;
  for (int64_t i = W * ((int64_t)blockIdx.x * 256 + threadIdx.x); i < n; i += (int64_t)gridDim.x * 256 * W) {
    Rows<W> qv, rv;
    qv.load_fs(q, fs, nfl, i);
    rv.load(r, i);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      rv.v[w] -= al * qv.v[w];
      acc += rv.v[w] * rv.v[w];
    }
    rv.store(r, i);
  }
  if (rr) {
    const double t = block_sum_tree(acc, sh);
    if (threadIdx.x == 0) rr[blockIdx.x] = t;
  }
}

// x += alpha p (x nullable), then pout = z + beta p (z unassembled; pout may
// be p itself): the solution update of an iteration rides on the direction
// update that reads p anyway.  With
// part: beta = rz_new / rz_old and the convergence test from the np partials
// of rz_new, reduced by every block in the same order; block 0 records them,
// counts the iteration and raises the flag, and every block of the
// iteration that converged returns without an update (the caller adds its
// x update afterwards).
template <int W>
__global__ __launch_bounds__(256) void k_xpay(double* __restrict__ x, const double* p, double* pout,
                                              const double* __restrict__ z, const double* __restrict__ fs,
                                              int64_t nfl, int64_t n, double* sc, int* flag,
                                              const double* __restrict__ part, int np) {
  __shared__ double sh[4];
  __shared__ int stop;
  // block 0 may raise the flag while other blocks start: each block reads it
  // once, so that the whole block takes one branch
  if (threadIdx.x == 0) stop = *flag;
  __syncthreads();
  if (stop) return;
  const double al = sc[SC_ALPHA];
  double be;
  if (part) {
    const double rz = block_sum_fixed(part, np, sh);
    be = rz / sc[SC_RZ_OLD];
    const bool conv = !(rz > sc[SC_TOL2]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[SC_BETA] = be;
      sc[SC_RZ] = rz;
      sc[SC_RES] = sc[SC_BPB] > 0 ? sqrt(fmax(rz, 0.0) / sc[SC_BPB]) : 0.0;
      flag[1] += 1;
      if (conv) flag[0] = 1;
    }
    if (conv) return;
  } else {
    be = sc[SC_BETA];
  }
  for (int64_t i = W * ((int64_t)blockIdx.x * 256 + threadIdx.x); i < n; i += (int64_t)gridDim.x * 256 * W) {
    Rows<W> pv, zv;
    pv.load(p, i);
    zv.load_fs(z, fs, nfl, i);
    if (x) {
      Rows<W> xv;
      xv.load(x, i);
#pragma unroll
      for (int w = 0; w < W; ++w) xv.v[w] += al * pv.v[w];
      xv.store(x, i);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) zv.v[w] += be * pv.v[w];
    zv.store(pout, i);
  }
}

// x += sum_{j < cnt} a_j p_j with p_j the ring slot (s0 + j) % H of hist
// ([H][n]) and a_j its alpha: the PCG solution update of cnt iterations in
// one pass, added in iteration order (the same roundings as one update per
// iteration).
template <int W>
__global__ __launch_bounds__(256) void k_xflush(double* __restrict__ x, const double* __restrict__ hist,
                                                const double* __restrict__ ahist, int64_t n, int H, int s0, int cnt) {
  for (int64_t i = W * ((int64_t)blockIdx.x * 256 + threadIdx.x); i < n; i += (int64_t)gridDim.x * 256 * W) {
    Rows<W> xv;
    xv.load(x, i);
    for (int j = 0; j < cnt; ++j) {
      const int slot = (s0 + j) % H;
      const double a = ahist[slot];
      Rows<W> pv;
      pv.load(hist + (int64_t)slot * n, i);
#pragma unroll
      for (int w = 0; w < W; ++w) xv.v[w] += a * pv.v[w];
    }
    xv.store(x, i);
  }
}

// r = b - q (q unassembled)
__global__ void k_sub_fs(double* __restrict__ r, const double* __restrict__ b, const double* __restrict__ q,
                         const double* __restrict__ fs, int64_t nfl, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    r[i] = b[i] - fs_row(q, fs, nfl, i);
}

__global__ void k_copy(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = x[i];
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] += a * x[i];
}

// w = a h1 + b h2 + c w (w may hold h3)
__global__ void k_comb3(double* __restrict__ w, const double* __restrict__ h1, const double* __restrict__ h2,
                        double a, double b, double c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    w[i] = a * h1[i] + b * h2[i] + (c != 0.0 ? c * w[i] : 0.0);
}

__global__ void k_copy_diag(double* dst, const double* sc, const int* flag) {
  dst[0] = (double)flag[1];
  dst[1] = sc[SC_RES];
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

void vec_dot(hipStream_t s, const double* a, const double* b, int64_t n, double* part, const int* flag) {
  hipLaunchKernelGGL(k_dot_partial, dim3(NPART), dim3(256), 0, s, a, b, n, part, flag);
}
void vec_scalar(hipStream_t s, const double* part, int np, double* sc, int* flag, int op, double arg,
                double* dst) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(256), 0, s, part, np, sc, flag, op, arg, dst);
}
static bool al16(const void* a) { return (reinterpret_cast<uintptr_t>(a) & 15) == 0; }
// at most 1024 blocks (four per CU): each block also reduces the scalar
// step's partials, and on the 7.9M-DoF workload 1024 beat 512 and 2048
static int grid_pairs(int64_t n) {
  const int64_t b = (n / 2 + 255) / 256;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

int vec_rupdate(hipStream_t s, double* r, const double* q, const double* fs, int64_t nfl, int64_t n, double* sc,
                const int* flag, const double* part, int np, double* rr, double* arec) {
  if (nfl % 2 == 0 && n % 2 == 0 && al16(r) && al16(q) && al16(fs)) {
    const int g = grid_pairs(n);
    hipLaunchKernelGGL((k_rupdate<2>), dim3(g), dim3(256), 0, s, r, q, fs, nfl, n, sc, flag, part, np, rr, arec);
    return g;
  }
  const int g = grid_for(n);
  hipLaunchKernelGGL((k_rupdate<1>), dim3(g), dim3(256), 0, s, r, q, fs, nfl, n, sc, flag, part, np, rr, arec);
  return g;
}
void vec_xpay(hipStream_t s, double* x, const double* p, double* pout, const double* z, const double* fs, int64_t nfl,
              int64_t n, double* sc, int* flag, const double* part, int np) {
  if (nfl % 2 == 0 && n % 2 == 0 && al16(x) && al16(p) && al16(pout) && al16(z) && al16(fs))
    hipLaunchKernelGGL((k_xpay<2>), dim3(grid_pairs(n)), dim3(256), 0, s, x, p, pout, z, fs, nfl, n, sc, flag, part,
                       np);
  else
    hipLaunchKernelGGL((k_xpay<1>), dim3(grid_for(n)), dim3(256), 0, s, x, p, pout, z, fs, nfl, n, sc, flag, part,
                       np);
}
void vec_xflush(hipStream_t s, double* x, const double* hist, const double* ahist, int64_t n, int H, int s0,
                int cnt) {
  if (cnt <= 0) return;
  if (n % 2 == 0 && al16(x) && al16(hist))
    hipLaunchKernelGGL((k_xflush<2>), dim3(grid_pairs(n)), dim3(256), 0, s, x, hist, ahist, n, H, s0, cnt);
  else
    hipLaunchKernelGGL((k_xflush<1>), dim3(grid_for(n)), dim3(256), 0, s, x, hist, ahist, n, H, s0, cnt);
}
void vec_sub_fs(hipStream_t s, double* r, const double* b, const double* q, const double* fs, int64_t nfl,
                int64_t n) {
  hipLaunchKernelGGL(k_sub_fs, dim3(grid_for(n)), dim3(256), 0, s, r, b, q, fs, nfl, n);
}
void vec_copy(hipStream_t s, double* y, const double* x, int64_t n) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, y, x, n);
}
void vec_axpy(hipStream_t s, double* y, const double* x, double a, int64_t n) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, y, x, a, n);
}
void vec_comb3(hipStream_t s, double* w, const double* h1, const double* h2, double a, double b, double c,
               int64_t n) {
  hipLaunchKernelGGL(k_comb3, dim3(grid_for(n)), dim3(256), 0, s, w, h1, h2, a, b, c, n);
}
void vec_copy_diag(hipStream_t s, double* dst, const double* sc, const int* flag) {
  hipLaunchKernelGGL(k_copy_diag, dim3(1), dim3(1), 0, s, dst, sc, flag);
}

}  // namespace hopu
