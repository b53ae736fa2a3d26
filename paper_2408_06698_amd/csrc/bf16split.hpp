// Split-BF16 contraction helpers of the element kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace hopu {

typedef float f4 __attribute__((ext_vector_type(4)));

// Split-BF16 contractions on the 16x16x16 BF16 MFMA with FP32 accumulation.
// Four consecutive K steps of the 16x16x4 FP32 form make one MFMA: register
// j of lane group g carries step 4s + j of that group on both operands, so
// the FP32 form's per-lane values and output layout (row 4g + i in register
// i) carry over unchanged, and the tables are the FP32 ones regrouped.  Each
// operand is split by truncation into NS bfloat16 terms (hi, [mid,] lo; each
// term the leading 8 bits of what the previous ones leave), and products two
// levels below the leading one or lower are dropped: NS = 2 keeps hh, hl,
// lh (each operand to about 16 significant bits, each product to about
// 13), NS = 3 keeps hh, hm, mh, hl, mm, lh (each FP32 operand exactly, each
// product to about 21 bits against FP32's 24).
template <int NS>
using BfTab = BfPack<(NS > 0 ? NS : 1)>;
template <typename T, int NS>
using TabT = std::conditional_t<NS == 0, T, BfTab<NS>>;

template <int NS>
__device__ __forceinline__ BfTab<NS> bf_split4(float b0, float b1, float b2, float b3) {
  BfTab<NS> p;
  const float v[4] = {b0, b1, b2, b3};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float r = v[j];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const uint32_t h = __float_as_uint(r) & 0xFFFF0000u;
      p.v[t][j] = (short)(h >> 16);
      r -= __uint_as_float(h);
    }
  }
  return p;
}

// steps s0 .. s0+3 of a lane's per-step values (zero past the end)
template <int NS, int N, typename T>
__device__ __forceinline__ BfTab<NS> bf_steps(const T (&b)[N], int s0) {
  return bf_split4<NS>(s0 < N ? (float)b[s0] : 0.f, s0 + 1 < N ? (float)b[s0 + 1] : 0.f,
                       s0 + 2 < N ? (float)b[s0 + 2] : 0.f, s0 + 3 < N ? (float)b[s0 + 3] : 0.f);
}

__device__ __forceinline__ f4 mfma_bf(bf16x4_t a, bf16x4_t b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// c += a b over one group of four steps, smaller products first
template <int NS>
__device__ __forceinline__ f4 mma_bf(const BfTab<NS>& a, const BfTab<NS>& b, f4 c) {
  if constexpr (NS == 2) {
    c = mfma_bf(a.v[1], b.v[0], c);
    c = mfma_bf(a.v[0], b.v[1], c);
  } else {
    c = mfma_bf(a.v[2], b.v[0], c);
    c = mfma_bf(a.v[1], b.v[1], c);
    c = mfma_bf(a.v[0], b.v[2], c);
    c = mfma_bf(a.v[1], b.v[0], c);
    c = mfma_bf(a.v[0], b.v[1], c);
  }
  return mfma_bf(a.v[0], b.v[0], c);
}

}  // namespace hopu
