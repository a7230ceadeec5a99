// Batched simplex lookup with the Pearson skill computed on the fly
// (kEDM paper: Section 2.1 steps 3-4, Section 3.4 and Algorithm 3).
//
// One workgroup takes one library table and a tile of T targets that share
// its embedding dimension.  The T target series are staged in LDS (only the
// window [t(0)+Tp, t(nq-1)+Tp] the table can touch), so every neighbour gather
// is an LDS read; each thread then walks query points p with a stride of 256,
// reads the table row of p once and reuses it for all T targets.  Predictions
// are written only on request; the co-moments of (observation, prediction)
// are accumulated per thread as shifted float64 sums and merged across the
// workgroup with the stable pairwise update, so rho needs no second pass.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

namespace edm {
namespace {

constexpr int kTMax = 8;               // targets per workgroup, upper bound
constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS for staged targets

template <int K>
__global__ __launch_bounds__(kLookupThreads) void k_lookup(LookupArgs a, int T, int slot0) {
  extern __shared__ float ys[];  // [T][m]
  __shared__ Mom wmom[kLookupThreads / kWave][kTMax];

  const int slot = slot0 + static_cast<int>(blockIdx.y);
  const int lib = a.lib_ids ? a.lib_ids[slot] : slot;
  const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
  const int off = (a.E - 1) * a.tau + a.Tp;
  const int m = static_cast<int>(Lx) - off;
  if (m - 1 < K) return;  // the table does not exist for this library
  const int t0 = static_cast<int>(blockIdx.x) * T;
  if (t0 >= a.ntgt) return;

  int tgt[kTMax];
  bool ok[kTMax];
  bool bad = false;
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    const int jt = t0 + t;
    ok[t] = t < T && jt < a.ntgt;
    tgt[t] = ok[t] ? (a.tgt_ids ? a.tgt_ids[jt] : jt) : 0;
    if (ok[t] && a.Ly_dev && a.Ly_dev[tgt[t]] < Lx) ok[t] = false;  // pair undefined
    if (ok[t]) {
      const float *__restrict__ y = a.Y + static_cast<int64_t>(tgt[t]) * a.ldy + off;
      for (int e = threadIdx.x; e < m; e += kLookupThreads) {
        const float v = y[e];
        bad |= !isfinite(v);
        ys[t * m + e] = v;
      }
    }
  }
  if (bad) atomicOr(a.status, 1);
  __syncthreads();

  double c = 0.0;
  double ro[kTMax], rp[kTMax], so[kTMax], sp[kTMax], soo[kTMax], spp[kTMax], sop[kTMax];
#pragma unroll
  for (int t = 0; t < kTMax; ++t) ro[t] = rp[t] = so[t] = sp[t] = soo[t] = spp[t] = sop[t] = 0.0;

  const int64_t tbl = static_cast<int64_t>(slot) * a.tbl_stride;
  for (int p = threadIdx.x; p < m; p += kLookupThreads) {
    int qi[K];
    float wi[K];
    const int64_t row = tbl + static_cast<int64_t>(p) * K;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      qi[i] = a.idx[row + i];
      wi[i] = a.w[row + i];
    }
#pragma unroll
    for (int t = 0; t < kTMax; ++t) {
      if (ok[t]) {
        // Predictions are accumulated relative to the target's first staged
        // sample c: sum_i w_i (y_i - c) equals Yhat - c because the weights
        // sum to one, and keeps the float32 error proportional to the
        // target's spread rather than its level.
        const float *yt = ys + t * m;
        const float ct = yt[0];
        float yh = 0.0f;
#pragma unroll
        for (int i = 0; i < K; ++i) yh = fmaf(wi[i], yt[qi[i]] - ct, yh);
        const double o = static_cast<double>(yt[p]) - static_cast<double>(ct);
        const double ph = static_cast<double>(yh);
        if (c == 0.0) {
          ro[t] = o;
          rp[t] = ph;
        }
        const double dO = o - ro[t], dP = ph - rp[t];
        so[t] += dO;
        sp[t] += dP;
        soo[t] += dO * dO;
        spp[t] += dP * dP;
        sop[t] += dO * dP;
        if (a.pred) a.pred[static_cast<int64_t>(tgt[t]) * a.ldpred + p] = yh + ct;
      }
    }
    c += 1.0;
  }

  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    if (t < T) {  // uniform
      const Mom mt = mom_wave_reduce(
          ok[t] ? mom_from_shifted_sums(c, ro[t], rp[t], so[t], sp[t], soo[t], spp[t], sop[t])
                : mom_zero());
      if (lane == 0) wmom[wave][t] = mt;
    }
  }
  __syncthreads();
  if (a.rho && static_cast<int>(threadIdx.x) < T) {
    const int t = threadIdx.x;
    const int jt = t0 + t;
    if (jt < a.ntgt) {
      Mom s = wmom[0][t];
#pragma unroll
      for (int w = 1; w < kLookupThreads / kWave; ++w) s = mom_merge(s, wmom[w][t]);
      const int j = a.tgt_ids ? a.tgt_ids[jt] : jt;
      const bool defined = !(a.Ly_dev && a.Ly_dev[j] < Lx);
      if (defined) a.rho[static_cast<int64_t>(lib) * a.ldrho + j] = static_cast<float>(mom_rho(s));
    }
  }
}

using LaunchFn = hipError_t (*)(const LookupArgs &, dim3, size_t, int, int, hipStream_t);

template <int K>
hipError_t launch_k(const LookupArgs &a, dim3 grid, size_t shm, int T, int slot0,
                    hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_lookup<K>);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_lookup<K>), grid, dim3(kLookupThreads), shm, st, a, T, slot0);
  return hipGetLastError();
}

template <size_t... I>
constexpr auto make_table(std::index_sequence<I...>) {
  return std::array<LaunchFn, sizeof...(I)>{&launch_k<static_cast<int>(I) + 1>...};
}

}  // namespace

hipError_t launch_lookup(const LookupArgs &a, int nslots, int64_t m_max, hipStream_t st) {
  static const auto table = make_table(std::make_index_sequence<EDM_K_MAX>{});
  if (nslots <= 0 || a.ntgt <= 0 || m_max <= 0) return hipSuccess;
  int T = static_cast<int>(kLdsBudget / (m_max * static_cast<int64_t>(sizeof(float))));
  if (T < 1) T = 1;
  if (T > kTMax) T = kTMax;
  if (T > a.ntgt) T = a.ntgt;
  const size_t shm = static_cast<size_t>(T) * static_cast<size_t>(m_max) * sizeof(float);
  const unsigned gx = static_cast<unsigned>((a.ntgt + T - 1) / T);
  constexpr int kMaxY = 32768;
  for (int s0 = 0; s0 < nslots; s0 += kMaxY) {
    const int ny = nslots - s0 < kMaxY ? nslots - s0 : kMaxY;
    hipError_t e = table[a.k - 1](a, dim3(gx, static_cast<unsigned>(ny)), shm, T, s0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace edm
