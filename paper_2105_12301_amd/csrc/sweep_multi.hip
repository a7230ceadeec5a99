// Batched E sweep: one candidate scan serves a whole group of embedding
// dimensions (kEDM paper: Section 2.1 steps 1-4 with E chosen empirically,
// Algorithms 1-2; the batching over E is this library's own).
//
// The ranking key of Algorithm 1 for dimension E is the float32 sum over the
// lags j < E in ascending order, so the key for E is exactly the key for E-1
// plus one more rounded term.  A lane that owns query p therefore walks its
// candidates once, extends the running sum lag by lag, and offers the partial
// sum to the top-k list of every E in its group as it passes: the tables (and
// so the correlations) are bit-identical to one scan per E, for
// 3*E_hi + (E_hi - E_lo + 1) VALU ops per pair instead of sum_E (3E + 1).
//
// Everything else follows the per-E kernel in knn.hip: library staged in LDS,
// one query per lane, diagonal candidate order (lane l sees q = s + l), a
// sliding window of samples in registers, insertions under a wave-uniform
// ballot, float64 weights of the winners, the self-prediction and its Pearson
// co-moments reduced per block.  tau = 1 only (the sweep's lag); other lags
// use the per-E kernel.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"
#include "scan_common.h"

#pragma clang fp contract(off)

namespace edm {
namespace {

constexpr int kUnroll = 8;

// One workgroup's share of a batched scan: query block `bx` of row `row`,
// every E in [ELO, EHI].  Called by the grid kernel and by the persistent
// kernel; every early return is uniform across the workgroup.
template <int ELO, int EHI>
__device__ __forceinline__ void group_scan(const KnnArgs &a, const int row, const int bx,
                                           float *__restrict__ xs) {
  constexpr int NG = EHI - ELO + 1;
  constexpr int TOT = list_off<ELO>(EHI + 1);
  __shared__ Mom wmom[kKnnThreads / kWave][NG];
  const uint32_t need = a.need_dev ? a.need_dev[row] : a.need;
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int Tp = a.Tp;
  // m(E) = queries = candidates at dimension E (tau = 1)
  const int m_lo = L - (ELO - 1) - Tp;
  const int m_hi = L - (EHI - 1) - Tp;
  if (m_lo - 1 < ELO + 1) return;  // no E of the group is feasible
  const int blk0 = bx * kKnnThreads;
  if (blk0 >= m_lo) return;

  bool bad = false;
  for (int i = threadIdx.x; i < L; i += kKnnThreads) {
    const float v = x[i];
    bad |= !isfinite(v);
    xs[i] = v;
  }
  if (bad) atomicOr(a.status, 1);
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform: readfirstlane lets the compiler keep it (and the self step) scalar
  const int p0 = __builtin_amdgcn_readfirstlane(blk0 + static_cast<int>(threadIdx.x & ~(kWave - 1)));
  const int p = p0 + lane;

  float vp[EHI];
#pragma unroll
  for (int j = 0; j < EHI; ++j) vp[j] = (p < m_lo && p + j < L) ? xs[p + j] : 0.0f;

  float qk[TOT];
  int qi[TOT];
  static_for<ELO, EHI>([&](auto EC) {
    constexpr int E = decltype(EC)::value;
    constexpr int OFF = list_off<ELO>(E);
    // table mode: lists of E that are not needed stay idle (kth = -1)
    const bool act = p < L - (E - 1) - Tp && (a.mom != nullptr || ((need >> (E - 1)) & 1u));
#pragma unroll
    for (int i = 0; i < E + 1; ++i) {
      qk[OFF + i] = act ? __builtin_inff() : -1.0f;
      qi[OFF + i] = -1;
    }
  });

  if (p0 < m_lo) {
    // Candidates whose window may run past some E's range: per-E validity.
    auto step_masked = [&](int s) {
      const int q = s + lane;
      const int qc = q < 0 ? 0 : q;
      float acc = 0.0f;
      static_for<0, EHI - 1>([&](auto JC) {
        constexpr int j = decltype(JC)::value;
        const int ix = qc + j < L ? qc + j : L - 1;
        const float d = vp[j] - xs[ix];
        acc = acc + d * d;
        if constexpr (j + 1 >= ELO) {
          constexpr int E = j + 1;
          const bool valid = q >= 0 && q < L - (E - 1) - Tp && s != p0;
          slice_offer<list_off<ELO>(E), E + 1, TOT>(qk, qi, acc, q, valid);
        }
      });
    };

    int s = -(kWave - 1);
#pragma unroll 1
    for (; s < 0; ++s) step_masked(s);
    const int s_full = m_hi - (kWave - 1);  // every lane's q < m_hi: valid for all E
    if (s + kUnroll <= s_full) {
      float win[EHI + kUnroll - 1];
#pragma unroll
      for (int j = 0; j < EHI - 1; ++j) win[j] = xs[s + lane + j];
      for (; s + kUnroll <= s_full; s += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) win[EHI - 1 + u] = xs[s + lane + EHI - 1 + u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const bool notself = s + u != p0;
          const int q = s + u + lane;
          float acc = 0.0f;
          float key[NG];
          static_for<0, EHI - 1>([&](auto JC) {
            constexpr int j = decltype(JC)::value;
            const float d = vp[j] - win[u + j];
            acc = acc + d * d;
            if constexpr (j + 1 >= ELO) key[j + 1 - ELO] = acc;
          });
          // One wave-uniform test for the whole group: some list improves iff
          // min over E of (key_E - kth_E) < 0 in some lane.  For finite keys
          // the sign of the float32 difference is exact; an empty list
          // (kth = +inf) gives -inf and an idle one (kth = -1) a positive
          // value.  The common step improves no list at all.
          if (notself) {
            float dm = key[0] - qk[list_off<ELO>(ELO) + ELO];
            static_for<ELO + 1, EHI>([&](auto EC) {
              constexpr int E = decltype(EC)::value;
              dm = fminf(dm, key[E - ELO] - qk[list_off<ELO>(E) + E]);
            });
            if (__builtin_amdgcn_ballot_w64(dm < 0.0f)) {
              static_for<ELO, EHI>([&](auto EC) {
                constexpr int E = decltype(EC)::value;
                slice_offer<list_off<ELO>(E), E + 1, TOT>(qk, qi, key[E - ELO], q, true);
              });
            }
          }
        }
#pragma unroll
        for (int j = 0; j < EHI - 1; ++j) win[j] = win[j + kUnroll];
      }
    }
#pragma unroll 1
    for (; s < m_lo; ++s) step_masked(s);
  }

  // Epilogue per E: float64 distances and weights of the winners, the
  // self-prediction Tp ahead, and the block's co-moments.
  const int wave = threadIdx.x / kWave;
  static_for<ELO, EHI>([&](auto EC) {
    constexpr int E = decltype(EC)::value;
    const Mom mine = finish_list<E, list_off<ELO>(E), TOT, EHI>(a, row, p, L, Tp, need, vp, qi, xs);
    if (a.mom) {  // uniform
      const Mom wv = mom_wave_reduce(mine);
      if (lane == 0) wmom[wave][E - ELO] = wv;
    }
  });
  if (a.mom == nullptr) return;
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < NG) {
    const int E = ELO + static_cast<int>(threadIdx.x);
    const int mE = L - (E - 1) - Tp;
    if (mE - 1 >= E + 1 && blk0 < mE) {
      Mom t = wmom[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kKnnThreads / kWave; ++w) t = mom_merge(t, wmom[w][threadIdx.x]);
      a.mom[(static_cast<int64_t>(row) * a.E_max + (E - 1)) * a.mom_blocks + bx] = t;
    }
  }
}

template <int ELO, int EHI>
__global__ __launch_bounds__(kKnnThreads) void k_sweep_multi(KnnArgs a, int slot0) {
  extern __shared__ float xs[];
  group_scan<ELO, EHI>(a, slot0 + static_cast<int>(blockIdx.y), static_cast<int>(blockIdx.x), xs);
}

// Persistent form: each workgroup pulls (row, block) items of one E group,
// ordered by the host longest first, from a device counter until the list is
// exhausted (every workgroup reaches the exit).  The item index travels
// through LDS and is made wave-uniform.
template <int ELO, int EHI>
__global__ __launch_bounds__(kKnnThreads) void k_tables_persistent(KnnArgs a,
                                                                   const TableItem *__restrict__ items,
                                                                   int n_items, int *counter) {
  extern __shared__ float xs[];
  __shared__ int item_s;
  for (int trip = 0;; ++trip) {  // one call site for the body (see lookup.hip)
    int it;
    if (counter == nullptr) {  // one item per workgroup
      if (trip > 0) break;
      it = static_cast<int>(blockIdx.x);
    } else {
      __syncthreads();  // the previous item is done with xs and item_s
      if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(item_s);
      if (it >= n_items) break;
    }
    const int row = __builtin_amdgcn_readfirstlane(items[it].row);
    const int blk = __builtin_amdgcn_readfirstlane(static_cast<int>(items[it].blk));
    group_scan<ELO, EHI>(a, row, blk, xs);
  }
}

// Groups of E sharing one scan: the register lists of a group hold at most
// ~54 entries (108 VGPRs).
constexpr int kGroups[][2] = {{1, 8}, {9, 12}, {13, 15}, {16, 18}, {19, 20}};

using LaunchFn = hipError_t (*)(const KnnArgs &, dim3, size_t, int, hipStream_t);

template <int ELO, int EHI>
hipError_t launch_group(const KnnArgs &a, dim3 grid, size_t shm, int slot0, hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_sweep_multi<ELO, EHI>);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_sweep_multi<ELO, EHI>), grid, dim3(kKnnThreads), shm, st, a, slot0);
  return hipGetLastError();
}

// table[lo-1][hi-lo]: every (lo, hi) with lo a group start and hi inside it.
template <int LO, size_t... I>
constexpr std::array<LaunchFn, 8> row_for(std::index_sequence<I...>) {
  return {{&launch_group<LO, LO + static_cast<int>(I)>...}};
}

}  // namespace

hipError_t launch_sweep_multi(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st) {
  static const std::array<LaunchFn, 8> t1 = row_for<1>(std::make_index_sequence<8>{});
  static const std::array<LaunchFn, 8> t9 = row_for<9>(std::make_index_sequence<4>{});
  static const std::array<LaunchFn, 8> t13 = row_for<13>(std::make_index_sequence<3>{});
  static const std::array<LaunchFn, 8> t16 = row_for<16>(std::make_index_sequence<3>{});
  static const std::array<LaunchFn, 8> t19 = row_for<19>(std::make_index_sequence<2>{});
  if (nslots <= 0) return hipSuccess;
  const unsigned gx = static_cast<unsigned>((L_max + kKnnThreads - 1) / kKnnThreads);
  const size_t shm = static_cast<size_t>(L_max) * sizeof(float);
  // With the matrix-core filter, E >= kGramEMin runs in the filtered groups.
  const bool gram = a.gram_nrm != nullptr && L_max <= kGramLMax;
  auto hi_of = [&](int lo, int top) {
    int hi = top < a.E_max ? top : a.E_max;
    if (a.mom == nullptr) {  // table mode: the group's scan must reach its largest needed E
      hi = 0;
      for (int E = lo; E <= top; ++E)
        if ((a.need >> (E - 1)) & 1u) hi = E;
    }
    return hi;
  };
  for (const auto &g : kGroups) {
    const int lo = g[0];
    if (gram && lo >= kGramEMin) break;
    const int hi = hi_of(lo, gram && g[1] >= kGramEMin ? kGramEMin - 1 : g[1]);
    if (hi == 0) continue;
    if (lo > hi) break;
    const std::array<LaunchFn, 8> &t = lo == 1 ? t1 : lo == 9 ? t9 : lo == 13 ? t13 : lo == 16 ? t16 : t19;
    LaunchFn fn = t[hi - lo];
    TimedLaunch timed(EDM_KF_BATCHED_SCAN, st);
    constexpr int kMaxY = 32768;
    for (int s0 = 0; s0 < nslots; s0 += kMaxY) {
      const int ny = nslots - s0 < kMaxY ? nslots - s0 : kMaxY;
      hipError_t e = fn(a, dim3(gx, static_cast<unsigned>(ny)), shm, s0, st);
      if (e != hipSuccess) return e;
    }
  }
  if (!gram) return hipSuccess;
  for (const auto &g : kGramGroups) {
    const int lo = g[0];
    const int hi = hi_of(lo, g[1]);
    if (hi == 0) continue;
    if (lo > hi) break;
    hipError_t e = launch_gram_group(a, lo, hi, nslots, L_max, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_tables_persistent(const KnnArgs &a, int group, const TableItem *items,
                                    int n_items, int *counter, int64_t L_max, int wg_per_cu,
                                    int n_cu, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  using Fn = void (*)(KnnArgs, const TableItem *, int, int *);
  // groups 0-4: the exact E groups; 5: E 1-4 (below the filtered groups)
  static const Fn fns[6] = {&k_tables_persistent<1, 8>, &k_tables_persistent<9, 12>,
                            &k_tables_persistent<13, 15>, &k_tables_persistent<16, 18>,
                            &k_tables_persistent<19, 20>, &k_tables_persistent<1, 4>};
  if (group < 0 || group > 5) return hipErrorInvalidValue;
  const size_t shm = static_cast<size_t>(L_max) * sizeof(float);
  const void *fn = reinterpret_cast<const void *>(fns[group]);
  TimedLaunch timed(EDM_KF_BATCHED_SCAN, st);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  if (wg_per_cu <= 0) {  // one workgroup per item
    hipLaunchKernelGGL(fns[group], dim3(static_cast<unsigned>(n_items)), dim3(kKnnThreads), shm, st,
                       a, items, n_items, static_cast<int *>(nullptr));
    return hipGetLastError();
  }
  int grid = wg_per_cu * n_cu;
  if (grid > n_items) grid = n_items;
  hipLaunchKernelGGL(fns[group], dim3(static_cast<unsigned>(grid)), dim3(kKnnThreads), shm, st, a,
                     items, n_items, counter);
  return hipGetLastError();
}

}  // namespace edm
