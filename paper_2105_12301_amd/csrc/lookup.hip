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
constexpr int kItemTMax = 4;           // the same for work-list items (register budget)
constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS for staged targets

// One workgroup's lookups: library `lib` with table (idx, w) [nq][K] at
// dimension E, targets tgt_ids[t0 .. t0+T) of a list of ntgt (identity list
// when tgt_ids is null).  Every early return is uniform across the workgroup.
template <int K, int kTMax>
__device__ __forceinline__ void lookup_body(const LookupArgs &a, const int E, const int lib,
                                            const int32_t *__restrict__ tidx,
                                            const float *__restrict__ tw,
                                            const int32_t *__restrict__ tgt_ids, const int t0,
                                            const int T, const int ntgt, float *__restrict__ ys) {
  __shared__ Mom wmom[kLookupThreads / kWave][kTMax];
  const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
  const int off = (E - 1) * a.tau + a.Tp;
  const int m = static_cast<int>(Lx) - off;
  if (m - 1 < K) return;  // the table does not exist for this library
  if (t0 >= ntgt) return;

  int tgt[kTMax];
  bool ok[kTMax];
  bool bad = false;
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    const int jt = t0 + t;
    ok[t] = t < T && jt < ntgt;
    tgt[t] = ok[t] ? (tgt_ids ? tgt_ids[jt] : jt) : 0;
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

  for (int p = threadIdx.x; p < m; p += kLookupThreads) {
    int qi[K];
    float wi[K];
    const int64_t row = static_cast<int64_t>(p) * K;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      qi[i] = tidx[row + i];
      wi[i] = tw[row + i];
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
    if (jt < ntgt) {
      Mom s = wmom[0][t];
#pragma unroll
      for (int w = 1; w < kLookupThreads / kWave; ++w) s = mom_merge(s, wmom[w][t]);
      const int j = tgt_ids ? tgt_ids[jt] : jt;
      const bool defined = !(a.Ly_dev && a.Ly_dev[j] < Lx);
      if (defined) a.rho[static_cast<int64_t>(lib) * a.ldrho + j] = static_cast<float>(mom_rho(s));
    }
  }
}

template <int K>
__global__ __launch_bounds__(kLookupThreads) void k_lookup(LookupArgs a, int T, int slot0) {
  extern __shared__ float ys[];  // [T][m]
  const int slot = slot0 + static_cast<int>(blockIdx.y);
  const int lib = a.lib_ids ? a.lib_ids[slot] : slot;
  const int64_t tbl = static_cast<int64_t>(slot) * a.tbl_stride;
  lookup_body<K, kTMax>(a, a.E, lib, a.idx + tbl, a.w + tbl, a.tgt_ids,
                        static_cast<int>(blockIdx.x) * T, T, a.ntgt, ys);
}

template <int K>
__device__ __forceinline__ void lookup_item(const LookupArgs &a, const LookupItem &w, float *ys) {
  const int64_t o = a.tbl_off[static_cast<int64_t>(w.lib) * (EDM_E_MAX + 1) + w.E];
  lookup_body<K, kItemTMax>(a, w.E, w.lib, a.tbl_idx + o, a.tbl_w + o,
                            a.bucket_ids + a.bucket_at[w.E], w.first, w.T, w.first + w.count, ys);
}

// Item kernel for one E (K = E + 1): persistent (counter != nullptr: loop
// pulling items) or one workgroup per item.  Item fields are made
// wave-uniform.
template <int K>
__global__ __launch_bounds__(kLookupThreads) void k_lookup_items(LookupArgs a,
                                                                const LookupItem *__restrict__ items,
                                                                int n_items, int *counter) {
  extern __shared__ float ys[];
  __shared__ int item_s;
  // One call site for the body (a second one would make the inliner emit a
  // real call with a scratch frame).  Without a counter each workgroup runs
  // the item of its own index once.
  for (int trip = 0;; ++trip) {
    int it;
    if (counter == nullptr) {
      if (trip > 0) break;
      it = static_cast<int>(blockIdx.x);
    } else {
      __syncthreads();
      if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(item_s);
      if (it >= n_items) break;
    }
    LookupItem w;
    w.lib = __builtin_amdgcn_readfirstlane(items[it].lib);
    w.E = static_cast<int16_t>(K - 1);
    w.T = static_cast<int16_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(items[it].T)));
    w.first = __builtin_amdgcn_readfirstlane(items[it].first);
    w.count = __builtin_amdgcn_readfirstlane(items[it].count);
    lookup_item<K>(a, w, ys);
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

hipError_t launch_lookup_items(const LookupArgs &a, int E, const LookupItem *items, int n_items,
                               int *counter, int64_t lds_floats, int wg_per_cu, int n_cu,
                               hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  using Fn = void (*)(LookupArgs, const LookupItem *, int, int *);
#define EDM_FN(E) &k_lookup_items<E + 1>
  static const Fn fns[EDM_E_MAX] = {EDM_FN(1),  EDM_FN(2),  EDM_FN(3),  EDM_FN(4),  EDM_FN(5),
                                    EDM_FN(6),  EDM_FN(7),  EDM_FN(8),  EDM_FN(9),  EDM_FN(10),
                                    EDM_FN(11), EDM_FN(12), EDM_FN(13), EDM_FN(14), EDM_FN(15),
                                    EDM_FN(16), EDM_FN(17), EDM_FN(18), EDM_FN(19), EDM_FN(20)};
#undef EDM_FN
  if (E < 1 || E > EDM_E_MAX) return hipErrorInvalidValue;
  const size_t shm = static_cast<size_t>(lds_floats) * sizeof(float);
  const void *fn = reinterpret_cast<const void *>(fns[E - 1]);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  if (wg_per_cu <= 0) {
    hipLaunchKernelGGL(fns[E - 1], dim3(static_cast<unsigned>(n_items)), dim3(kLookupThreads), shm,
                       st, a, items, n_items, static_cast<int *>(nullptr));
  } else {
    int grid = wg_per_cu * n_cu;
    if (grid > n_items) grid = n_items;
    hipLaunchKernelGGL(fns[E - 1], dim3(static_cast<unsigned>(grid)), dim3(kLookupThreads), shm, st,
                       a, items, n_items, counter);
  }
  return hipGetLastError();
}

}  // namespace edm
