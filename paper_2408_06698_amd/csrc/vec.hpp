#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hopu {
enum { NPART = 1024 };
enum { SC_RZ = 0, SC_ALPHA = 1, SC_BETA = 2, SC_TOL2 = 3, SC_BPB = 4, SC_RES = 5, SC_RZ_OLD = 6, SC_N = 8 };
enum { OP_SET_TOL = 0, OP_SET_RZ = 1, OP_STORE = 4, OP_STORE_SQRT = 5 };
void vec_dot(hipStream_t s, const double* a, const double* b, int64_t n, double* part, const int* flag);
void vec_scalar(hipStream_t s, const double* part, int np, double* sc, int* flag, int op, double arg,
                double* dst);
// q, z, and q in vec_sub_fs are unassembled: facet rows [0, nfl) come from the
// facet-side buffer fs ([2][nfl]), interior rows from the vector itself.
// PCG updates: r -= alpha q; then x += alpha p, p = z + beta p.  The
// scalar steps ride on the updates: vec_rupdate takes alpha = rz / (p.q)
// from the np partials of p.q (part, from the operator launch before it),
// records it in *arec if given and, if rr is given, leaves one partial of
// r.r per block there (returns the block count); vec_xpay takes beta and
// the convergence test from the np partials of the new rz, counts the
// iteration in flag[1] and raises flag[0] on convergence; it writes
// z + beta p to pout (may be p) and, if x is given, adds alpha p to it.
// part == nullptr: alpha / beta are read from sc as they are.  vec_xflush
// adds cnt recorded directions to x in order:
// x += sum_j ahist[(s0+j)%H] hist[(s0+j)%H][.] (hist [H][n]).
int vec_rupdate(hipStream_t s, double* r, const double* q, const double* fs, int64_t nfl, int64_t n, double* sc,
                const int* flag, const double* part, int np, double* rr, double* arec = nullptr);
void vec_xpay(hipStream_t s, double* x, const double* p, double* pout, const double* z, const double* fs, int64_t nfl,
              int64_t n, double* sc, int* flag, const double* part, int np);
void vec_xflush(hipStream_t s, double* x, const double* hist, const double* ahist, int64_t n, int H, int s0,
                int cnt);
void vec_sub_fs(hipStream_t s, double* r, const double* b, const double* q, const double* fs, int64_t nfl,
                int64_t n);
void vec_copy(hipStream_t s, double* y, const double* x, int64_t n);
void vec_axpy(hipStream_t s, double* y, const double* x, double a, int64_t n);
void vec_comb3(hipStream_t s, double* w, const double* h1, const double* h2, double a, double b, double c,
               int64_t n);
void vec_copy_diag(hipStream_t s, double* dst, const double* sc, const int* flag);
}  // namespace hopu
