// Batched simplex lookup with the Pearson skill computed on the fly
// (kEDM paper: Section 2.1 steps 3-4, Section 3.4 and Algorithm 3).
//
// A (library, target) pair is computed by one wave: its lanes walk the query
// points p = lane, lane + 64, ..., read the table row of p (K indices and
// weights), gather the K neighbours' futures of the target from LDS, and
// accumulate float64 sums of the observation and the prediction, both
// relative to the target's first staged sample (the weights sum to one, so
// the prediction minus that sample is the weighted sum of the gathered
// samples minus it; the float32 error stays proportional to the target's
// spread).  The sums are reduced over the wave by a fixed butterfly, so a
// pair's result does not depend on which kernel computed it or on how many
// targets share the wave: the grid kernel, the work-list kernel of the plan
// and every form are bit-identical.
//
// Grid kernel: a workgroup stages a tile of T targets of one E (the window
// [t(0)+Tp, t(nq-1)+Tp] the tables can touch) and its 8 waves run 8
// libraries' tables against them, each wave reusing every table row for the
// T targets (8 waves: two workgroups of 64 KB staging fill a CU with 16
// waves).  Work-list kernel: one item (a group of up to 16 libraries of
// similar length, T <= 16 targets staged in up to 160 KB) per workgroup of 16
// waves; wave w runs library w against the staged targets, reusing each table
// row for up to 4 targets.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

namespace edm {
namespace {

constexpr int kTMax = 8;               // targets per grid workgroup, upper bound
constexpr int kItemTMax = kLookupItemMaxTargets;
// Work-list kernel: one wave per library of an item, so every CU keeps 16
// waves busy however few targets of a long series fit its LDS.
constexpr int kItemThreads = kLookupItemLibs * 64;
// targets per table pass of a wave (fewer for the widest rows: registers)
template <int K>
constexpr int wave_targets() {
  return K <= 20 ? 4 : 2;
}
constexpr int kGridWaves = 8;  // libraries per grid workgroup (one wave each)
constexpr int kGridThreads = kGridWaves * kWave;
constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS for staged targets

struct Sums {
  double so, sp, soo, spp, sop;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Skill sums of one wave for TW targets (ok[t] false: skipped) through the
// table (tidx, tw) [m][K].  yt[t]: the target's staged window in LDS.
// pred[t] (or null): prediction output row.
template <int K, int TW>
__device__ __forceinline__ void wave_pairs(const int32_t *__restrict__ tidx,
                                           const float *__restrict__ tw, const int m,
                                           const float *const (&yt)[TW], const bool (&ok)[TW],
                                           float *const (&pred)[TW], Sums (&s)[TW]) {
  const int lane = threadIdx.x & (kWave - 1);
  float ct[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    s[t] = Sums{0.0, 0.0, 0.0, 0.0, 0.0};
    ct[t] = ok[t] ? yt[t][0] : 0.0f;
  }
  for (int p = lane; p < m; p += kWave) {
    int qi[K];
    float wi[K];
    const int64_t row = static_cast<int64_t>(p) * K;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      qi[i] = tidx[row + i];
      wi[i] = tw[row + i];
    }
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      if (ok[t]) {
        const float *y = yt[t];
        float yh = 0.0f;
#pragma unroll
        for (int i = 0; i < K; ++i) yh = fmaf(wi[i], y[qi[i]] - ct[t], yh);
        const double o = static_cast<double>(y[p]) - static_cast<double>(ct[t]);
        const double ph = static_cast<double>(yh);
        // explicit fused forms: the same operations in every instantiation
        s[t].so += o;
        s[t].sp += ph;
        s[t].soo = fma(o, o, s[t].soo);
        s[t].spp = fma(ph, ph, s[t].spp);
        s[t].sop = fma(o, ph, s[t].sop);
        if (pred[t]) pred[t][p] = yh + ct[t];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    if (ok[t]) {  // uniform across the wave
      s[t].so = wave_sum(s[t].so);
      s[t].sp = wave_sum(s[t].sp);
      s[t].soo = wave_sum(s[t].soo);
      s[t].spp = wave_sum(s[t].spp);
      s[t].sop = wave_sum(s[t].sop);
    }
  }
}

__device__ __forceinline__ float pair_rho(int m, const Sums &s) {
  return static_cast<float>(
      mom_rho(mom_from_shifted_sums(static_cast<double>(m), 0.0, 0.0, s.so, s.sp, s.soo, s.spp, s.sop)));
}

// Stage the window [off, off + n) of T targets into ys[t * ms + e], zero past
// a target's own length.
__device__ __forceinline__ void stage_targets(const LookupArgs &a, const int *tgt, int T, int off,
                                              int n, int ms, float *ys) {
  bool bad = false;
  for (int t = 0; t < T; ++t) {
    const int64_t Ly = a.Ly_dev ? a.Ly_dev[tgt[t]] : a.ldy;
    const int n_t = static_cast<int>(Ly - off < n ? Ly - off : n);
    const float *__restrict__ y = a.Y + static_cast<int64_t>(tgt[t]) * a.ldy + off;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      float v = 0.0f;
      if (e < n_t) {
        v = y[e];
        bad |= !isfinite(v);
      }
      ys[t * ms + e] = v;
    }
  }
  if (bad) atomicOr(a.status, 1);
}

// Grid kernel: blockIdx.x = tile of T targets, blockIdx.y = group of
// kGridWaves library slots; ms = LDS row stride (>= every staged window).
template <int K>
__global__ __launch_bounds__(kGridThreads) void k_lookup(LookupArgs a, int T, int ms,
                                                           int nslots, int slot0) {
  extern __shared__ float ys[];  // [T][ms]
  const int t0 = static_cast<int>(blockIdx.x) * T;
  const int sbase = slot0 + static_cast<int>(blockIdx.y) * kGridWaves;
  const int off = (a.E - 1) * a.tau + a.Tp;
  int tgt[kTMax];
  const int Tn = a.ntgt - t0 < T ? a.ntgt - t0 : T;
#pragma unroll
  for (int t = 0; t < kTMax; ++t) tgt[t] = t < Tn ? (a.tgt_ids ? a.tgt_ids[t0 + t] : t0 + t) : 0;
  int n_blk = 0;  // widest query range of the workgroup's libraries
  for (int w = 0; w < kGridWaves; ++w) {
    const int slot = sbase + w;
    if (slot >= slot0 + nslots) break;
    const int lib = a.lib_ids ? a.lib_ids[slot] : slot;
    const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
    const int mw = static_cast<int>(Lx) - off;
    n_blk = mw > n_blk ? mw : n_blk;
  }
  if (n_blk - 1 < K) return;  // no table in this workgroup (uniform)
  stage_targets(a, tgt, Tn, off, n_blk, ms, ys);
  __syncthreads();

  const int wave = static_cast<int>(threadIdx.x) / kWave;
  const int slot = __builtin_amdgcn_readfirstlane(sbase + wave);
  if (slot >= slot0 + nslots) return;
  const int lib = a.lib_ids ? a.lib_ids[slot] : slot;
  const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
  const int m = static_cast<int>(Lx) - off;
  if (m - 1 < K) return;  // the table does not exist for this library
  const int64_t tbl = static_cast<int64_t>(slot) * a.tbl_stride;
  const float *yt[kTMax];
  bool ok[kTMax];
  float *pred[kTMax];
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    yt[t] = ys + t * ms;
    ok[t] = t < Tn && !(a.Ly_dev && a.Ly_dev[tgt[t]] < Lx);  // pair defined
    pred[t] = (ok[t] && a.pred) ? a.pred + static_cast<int64_t>(tgt[t]) * a.ldpred : nullptr;
  }
  Sums s[kTMax];
  wave_pairs<K, kTMax>(a.idx + tbl, a.w + tbl, m, yt, ok, pred, s);
  if (a.rho && (threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int t = 0; t < kTMax; ++t)
      if (ok[t]) a.rho[static_cast<int64_t>(lib) * a.ldrho + tgt[t]] = pair_rho(m, s[t]);
  }
}

// Work-list kernel for one E (K = E + 1): persistent (counter != nullptr:
// workgroups pull items) or one workgroup per item.  An item stages a tile of
// targets once, over the window of its longest library, and wave w runs the
// item's library w against every staged target, kWaveT targets per table
// pass.  Item fields are made wave-uniform.
template <int K>
__global__ __launch_bounds__(kItemThreads) void k_lookup_items(LookupArgs a,
                                                                const LookupItem *__restrict__ items,
                                                                int n_items, int *counter) {
  extern __shared__ float ys[];
  __shared__ int item_s;
  __shared__ int tgt[kItemTMax];
  constexpr int kWaveT = wave_targets<K>();
  const int E = K - 1;
  const int off = (E - 1) * a.tau + a.Tp;
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  for (int trip = 0;; ++trip) {
    int it;
    if (counter == nullptr) {
      if (trip > 0) break;
      it = static_cast<int>(blockIdx.x);
    } else {
      __syncthreads();  // the previous item is done with ys, tgt and item_s
      if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(item_s);
      if (it >= n_items) break;
    }
    const int at = __builtin_amdgcn_readfirstlane(items[it].lib);
    const int nlib = __builtin_amdgcn_readfirstlane(static_cast<int>(items[it].nlib));
    const int T = __builtin_amdgcn_readfirstlane(static_cast<int>(items[it].T));
    const int first = __builtin_amdgcn_readfirstlane(items[it].first);
    const int count = __builtin_amdgcn_readfirstlane(items[it].count);
    const int Tn = count < T ? count : T;
    // the first library of an item is its longest: its window covers all
    const int lib0 = __builtin_amdgcn_readfirstlane(a.item_libs[at]);
    const int ms = static_cast<int>((a.Lx_dev ? a.Lx_dev[lib0] : a.Lx_uni) - off);
    if (static_cast<int>(threadIdx.x) < Tn) tgt[threadIdx.x] = a.bucket_ids[a.bucket_at[E] + first + threadIdx.x];
    __syncthreads();
    if (ms >= 1) stage_targets(a, tgt, Tn, off, ms, ms, ys);
    __syncthreads();
    if (wave < nlib) {  // uniform per wave
      const int lib = __builtin_amdgcn_readfirstlane(a.item_libs[at + wave]);
      const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
      const int m = static_cast<int>(Lx) - off;
      if (m - 1 >= K) {
        const int64_t o = a.tbl_off[static_cast<int64_t>(lib) * (EDM_E_MAX + 1) + E];
        for (int t0 = 0; t0 < Tn; t0 += kWaveT) {
          const float *yt[kWaveT];
          bool ok[kWaveT];
          float *pred[kWaveT];
          int id[kWaveT];
#pragma unroll
          for (int u = 0; u < kWaveT; ++u) {
            const int t = t0 + u;
            id[u] = tgt[t < Tn ? t : 0];
            yt[u] = ys + (t < Tn ? t : 0) * ms;
            ok[u] = t < Tn && !(a.Ly_dev && a.Ly_dev[id[u]] < Lx);
            pred[u] = nullptr;
          }
          Sums s[kWaveT];
          wave_pairs<K, kWaveT>(a.tbl_idx + o, a.tbl_w + o, m, yt, ok, pred, s);
          if (a.rho && (threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
            for (int u = 0; u < kWaveT; ++u)
              if (ok[u]) a.rho[static_cast<int64_t>(lib) * a.ldrho + id[u]] = pair_rho(m, s[u]);
          }
        }
      }
    }
  }
}

using LaunchFn = hipError_t (*)(const LookupArgs &, dim3, size_t, int, int, int, int, hipStream_t);

template <int K>
hipError_t launch_k(const LookupArgs &a, dim3 grid, size_t shm, int T, int ms, int nslots,
                    int slot0, hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_lookup<K>);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_lookup<K>), grid, dim3(kGridThreads), shm, st, a, T, ms, nslots, slot0);
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
  const int ms = static_cast<int>(m_max);
  const size_t shm = static_cast<size_t>(T) * static_cast<size_t>(m_max) * sizeof(float);
  const unsigned gx = static_cast<unsigned>((a.ntgt + T - 1) / T);
  constexpr int kMaxY = 32768 * kGridWaves;
  for (int s0 = 0; s0 < nslots; s0 += kMaxY) {
    const int ns = nslots - s0 < kMaxY ? nslots - s0 : kMaxY;
    const unsigned gy = static_cast<unsigned>((ns + kGridWaves - 1) / kGridWaves);
    hipError_t e = table[a.k - 1](a, dim3(gx, gy), shm, T, ms, ns, s0, st);
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
    hipLaunchKernelGGL(fns[E - 1], dim3(static_cast<unsigned>(n_items)), dim3(kItemThreads), shm,
                       st, a, items, n_items, static_cast<int *>(nullptr));
  } else {
    int grid = wg_per_cu * n_cu;
    if (grid > n_items) grid = n_items;
    hipLaunchKernelGGL(fns[E - 1], dim3(static_cast<unsigned>(grid)), dim3(kItemThreads), shm, st,
                       a, items, n_items, counter);
  }
  return hipGetLastError();
}

}  // namespace edm
