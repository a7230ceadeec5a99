// Register top-k lists and the per-E epilogue shared by the batched scans
// (exact VALU scan in sweep_multi.hip, matrix-core filter in gram.hip).
// Every file that includes this header is compiled with FP contraction off.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

namespace edm {

template <int I0, int I1, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I0 <= I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

// Offset of dimension E's list inside the flat register arrays of a group
// whose smallest dimension is ELO (list of E holds E + 1 entries).
template <int ELO>
constexpr int list_off(int E) {
  int o = 0;
  for (int e = ELO; e < E; ++e) o += e + 1;
  return o;
}

// Sorted insertion into the slice [OFF, OFF+K) of the flat lists.  A lane's
// candidates arrive in ascending q, so the strict comparisons keep equal keys
// in index order; inserting +inf (or any key not below the last entry) leaves
// the slice unchanged, which lets a whole wave run it without lane masking.
template <int OFF, int K, int TOT>
__device__ __forceinline__ void slice_insert(float (&qk)[TOT], int (&qi)[TOT], float key, int q) {
#pragma unroll
  for (int i = K - 1; i > 0; --i) {
    const bool lt_prev = key < qk[OFF + i - 1];
    const bool lt_cur = key < qk[OFF + i];
    qi[OFF + i] = lt_prev ? qi[OFF + i - 1] : (lt_cur ? q : qi[OFF + i]);
    qk[OFF + i] = __builtin_amdgcn_fmed3f(qk[OFF + i - 1], key, qk[OFF + i]);
  }
  const bool lt0 = key < qk[OFF];
  qi[OFF] = lt0 ? q : qi[OFF];
  qk[OFF] = lt0 ? key : qk[OFF];
}

template <int OFF, int K, int TOT>
__device__ __forceinline__ void slice_offer(float (&qk)[TOT], int (&qi)[TOT], float key, int q,
                                            bool valid) {
  const bool want = valid && key < qk[OFF + K - 1];
  if (__builtin_amdgcn_ballot_w64(want))
    slice_insert<OFF, K, TOT>(qk, qi, want ? key : __builtin_inff(), q);
}

// Final step for dimension E of query p: float64 distances and weights of the
// K = E + 1 winners (Section 2.1 step 3, "Normalize D_k" of Algorithm 2),
// then either the table row (table mode) or the query's self-prediction Tp
// ahead (sweep mode, returned as a one-point moment).  vp holds the query's
// samples, xs the staged series.  The list slice is consumed.
template <int E, int OFF, int TOT, int NV>
__device__ __forceinline__ Mom finish_list(const KnnArgs &a, int row, int p, int L, int Tp,
                                           uint32_t need, const float (&vp)[NV],
                                           int (&qi)[TOT], const float *__restrict__ xs) {
  constexpr int K = E + 1;
  const int mE = L - (E - 1) - Tp;
  Mom mine = mom_zero();
  const bool want_table = a.mom == nullptr && ((need >> (E - 1)) & 1u);
  if (p < mE && mE - 1 >= K && (a.mom != nullptr || want_table)) {
    double D[K];
    double dmin = __builtin_inf();
#pragma unroll 1
    for (int r = 0; r < K; ++r) {
      const int q = qi[OFF] < 0 ? 0 : qi[OFF];
      double s2 = 0.0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const double d = static_cast<double>(vp[j]) - static_cast<double>(xs[q + j]);
        s2 += d * d;
      }
      const double dq = sqrt(s2);
      dmin = fmin(dmin, dq);
#pragma unroll
      for (int i = 0; i < K - 1; ++i) {
        qi[OFF + i] = qi[OFF + i + 1];
        D[i] = D[i + 1];
      }
      qi[OFF + K - 1] = q;
      D[K - 1] = dq;
    }
    double wsum = 0.0;
#pragma unroll 1
    for (int r = 0; r < K; ++r) {
      const double d = D[0];
      const double wq = dmin > 0.0 ? exp(-d / dmin) : (d == 0.0 ? 1.0 : 0.0);
      wsum += wq;
#pragma unroll
      for (int i = 0; i < K - 1; ++i) D[i] = D[i + 1];
      D[K - 1] = wq;
    }
    const double inv = 1.0 / wsum;
    if (want_table) {
      int32_t *ti;
      float *tw;
      int64_t base;
      if (a.tbl_off) {
        const int64_t o = a.tbl_off[static_cast<int64_t>(row) * (EDM_E_MAX + 1) + E];
        ti = a.tbl_idx + o;
        tw = a.tbl_w + o;
        base = static_cast<int64_t>(p) * K;
      } else {
        ti = a.idxE[E];
        tw = a.wE[E];
        base = static_cast<int64_t>(row) * a.strideE[E] + static_cast<int64_t>(p) * K;
      }
#pragma unroll
      for (int i = 0; i < K; ++i) {
        ti[base + i] = qi[OFF + i];
        tw[base + i] = static_cast<float>(D[i] * inv);
      }
    } else {
      if (a.keepE[E]) {  // sweep mode: keep the sorted list for a later cross map
        const int64_t ko = static_cast<int64_t>(row) * a.keep_strideE[E] + static_cast<int64_t>(p) * K;
#pragma unroll
        for (int i = 0; i < K; ++i) a.keepE[E][ko + i] = qi[OFF + i];
        if (a.keepWE[E]) {
#pragma unroll
          for (int i = 0; i < K; ++i) a.keepWE[E][ko + i] = static_cast<float>(D[i] * inv);
        }
      }
      const int o_off = (E - 1) + Tp;
      double yh = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i) yh += (D[i] * inv) * static_cast<double>(xs[qi[OFF + i] + o_off]);
      mine.n = 1.0;
      mine.mo = static_cast<double>(xs[p + o_off]);
      mine.mp = yh;
    }
  }
  return mine;
}

}  // namespace edm
