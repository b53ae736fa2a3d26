// Device kernels of the HOPU convection library (gfx950 / CDNA4).
// One wave64 owns a batch of 16 elements; every basis contraction is a
// 16x16x4 MFMA whose N dimension runs over those elements.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.hpp"

namespace hopu {

template <int D, int KK>
struct Cfg {
  static constexpr int NP = D == 2 ? (KK + 1) * (KK + 2) / 2 : (KK + 1) * (KK + 2) * (KK + 3) / 6;
  static constexpr int NPS = (NP + 3) / 4 * 4;
  static constexpr int NM = D * NPS;
  static constexpr int N = D * NP;
  static constexpr int NF = D == 2 ? KK + 1 : (KK + 1) * (KK + 2) / 2;
  static constexpr int NFL = (D + 1) * NF;
  static constexpr int NINT = N - NFL;
  static constexpr int PV = (3 * KK + 1) / 2;
  static constexpr int PF = (3 * KK + 2) / 2;
  static constexpr int NQV = D == 2 ? PV * PV : PV * PV * PV;
  static constexpr int NQF = D == 2 ? PF : PF * PF;
  static constexpr int NMT = (NM + 15) / 16;
  static constexpr int NK = (N + 3) / 4;
  static constexpr int NQVT = (NQV + 15) / 16;
  static constexpr int NPK = NPS / 4;
  static constexpr int NAT = (NP + 15) / 16;
  static constexpr int NQFT = (NQF + 15) / 16;
  static constexpr int NFJT = (NF + 15) / 16;
  static constexpr int NFK = 4 * NFJT;
  static constexpr int NJT = (N + 15) / 16;
  static constexpr int NMQ = 4 * NMT;
  // projection step: dim P^{k-1}
  static constexpr int NQ = D == 2 ? KK * (KK + 1) / 2 : KK * (KK + 1) * (KK + 2) / 6;
};


// Split-BF16 fragment of a 16x16x16 BF16 MFMA operand: a lane's four K
// values as NS bfloat16 terms (hi, [mid,] lo) whose sum is the FP32 value
// to 8 NS significant bits (raw bfloat16 bits).
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
template <int NS>
struct BfPack {
  bf16x4_t v[NS];
};

// Device pointers to one precision's fragment tables and weights.
template <typename T>
struct DevTables {
  const T* modal;
  const T* vol_V;
  const T* vol_dVT;
  const T* vol_dV;
  const T* vol_VT;
  const T* fac_Tr;
  const T* fac_TrT;
  const T* fac_K;
  const T* fac_Psi;
  const T* fac_PsiT;
  const T* fac_KT;
  const T* dual;
  const double* dual64;  // reduced forms: FP64 values of `dual` in their K order
  const double* wv;
  const double* wf;
  const int* psi_deg;
};

// The dual-transform table in FP64 (the transform runs in FP64 in every form).
__host__ __device__ inline const double* dual_f64(const DevTables<double>& t) { return t.dual; }
template <typename T>
__host__ __device__ inline const double* dual_f64(const DevTables<T>& t) {
  return t.dual64;
}

struct DevMesh {
  const double* geo;
  const int32_t* fid;
  const int32_t* nbr;
  const int32_t* facet_elem;
  const int8_t* facet_local;
  const int8_t* fside;  // [E][d+1]: 0 if the element is facet_elem[2F] on that side, else 1
  const int32_t* belem;
  const int32_t* bsig;
  const int8_t* lfac;  // nullable
  int64_t E, F, nb;
  int lglob;
};

}  // namespace hopu
