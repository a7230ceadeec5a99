// All k-nearest-neighbour tables, fused with the time-delay embedding and the
// simplex weights (kEDM paper: Section 2.1 steps 1-3, Algorithms 1 and 2).
//
// Design for gfx950
// -----------------
// * The paper materialises the L x L distance matrix (Algorithm 1) and then
//   partially sorts each row (Algorithm 2).  Here nothing of size L^2 ever
//   leaves the compute unit: each workgroup stages its library series once in
//   LDS (<= 128 KiB of the 160 KiB per CU), each lane owns one query point,
//   keeps its E coordinates and its sorted top-k (key, index) list in VGPRs,
//   and streams every candidate through them.  The embedding is never stored
//   (Section 3.3.1 fuses it for the same reason).
// * Diagonal scan: at step s, lane l of a wave whose queries are p0..p0+63
//   evaluates candidate q = s + l.  Consecutive queries have time-shifted
//   neighbourhoods (v_{p+1} shares E-1 coordinates with v_p), so their top-k
//   insertions fall on the same step and the wave diverges far less often
//   than with every lane looking at the same candidate.  Every lane still
//   visits its candidates in ascending q, so a strict "<" keeps equal keys in
//   index order (ties broken by the lower index), and the self step q = p is
//   the same step s = p0 for the whole wave (as is every step of an
//   exclusion window |q - p| <= r: q - p = s - p0 for every lane).
// * tau = 1: each lane keeps a sliding window of E + U - 1 samples in
//   registers and loads one new LDS word per candidate, so the key costs
//   exactly E subtractions, E multiplies and E adds of float32 VALU work.
// * The ranking key is the float32 sum of Algorithm 1 in lag order with a
//   rounding after every operation: this file is compiled with contraction off
//   (and says so with a pragma), and fp32 denormals are kept (gfx950 default).
// * Weights need only the k winners: their distances are recomputed in
//   float64 from the staged samples, w_i = exp(-d_i / d_min) normalised
//   (Section 2.1 step 3, "Normalize D_k" in Algorithm 2).
// * Sweep mode fuses the self-prediction and its Pearson co-moments into the
//   epilogue, so the E sweep writes no table at all.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

#pragma clang fp contract(off)

namespace edm {
namespace {

constexpr int kUnroll = 8;

// Sorted insertion of (key, q) into the ascending list qk/qi held in
// registers.  A lane's candidates arrive in ascending q, so the strict
// comparisons keep equal keys in index order.  Inserting +inf (or any key not
// below qk[K-1]) leaves the list unchanged, which lets a whole wave run the
// insertion without lane masking.
template <int K>
__device__ __forceinline__ void topk_insert(float (&qk)[K], int (&qi)[K], float key, int q) {
#pragma unroll
  for (int i = K - 1; i > 0; --i) {
    const bool lt_prev = key < qk[i - 1];
    const bool lt_cur = key < qk[i];
    qi[i] = lt_prev ? qi[i - 1] : (lt_cur ? q : qi[i]);
    // qk[i-1] <= qk[i], so the median is the new value of slot i.
    qk[i] = __builtin_amdgcn_fmed3f(qk[i - 1], key, qk[i]);
  }
  const bool lt0 = key < qk[0];
  qi[0] = lt0 ? q : qi[0];
  qk[0] = lt0 ? key : qk[0];
}

// Offer (key, q) to the lane's list.  The insertion runs only when at least
// one lane of the wave improves its list (a wave-uniform branch), which after
// the first few hundred candidates is rare.
template <int K>
__device__ __forceinline__ void topk_offer(float (&qk)[K], int (&qi)[K], float key, int q,
                                           bool valid) {
  const bool want = valid && key < qk[K - 1];
  if (__builtin_amdgcn_ballot_w64(want)) topk_insert<K>(qk, qi, want ? key : __builtin_inff(), q);
}

template <int E_T, int K, bool T1>
__global__ __launch_bounds__(kKnnThreads) void k_knn(KnnArgs a, int slot0) {
  constexpr int EM = E_T ? E_T : EDM_E_MAX;
  extern __shared__ float xs[];
  __shared__ Mom wmom[kKnnThreads / kWave];

  const int slot = slot0 + static_cast<int>(blockIdx.y);
  const int row = a.lib_ids ? a.lib_ids[slot] : slot;
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int E = E_T ? E_T : a.E;
  const int tau = T1 ? 1 : a.tau;
  const int off = (E - 1) * tau;
  const int m = L - off - a.Tp;  // queries = candidates
  const int excl = a.excl;       // exclusion radius: |q - p| <= excl is no candidate
  if (m - 1 - 2 * excl < K) return;  // infeasible for this series (uniform)
  const int blk0 = static_cast<int>(blockIdx.x) * kKnnThreads;
  if (blk0 >= m) return;

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
  const bool active = p < m;

  float vp[EM];
#pragma unroll
  for (int j = 0; j < EM; ++j) vp[j] = (active && (E_T || j < E)) ? xs[p + j * tau] : 0.0f;

  float qk[K];
  int qi[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    qk[i] = active ? __builtin_inff() : -1.0f;  // -1: an idle lane never inserts
    qi[i] = -1;
  }

  if (p0 < m) {  // wave-uniform: a wave with no query skips the scan
    auto step_masked = [&](int s) {
      const int q = s + lane;
      const bool valid = static_cast<unsigned>(q) < static_cast<unsigned>(m);
      const int qc = valid ? q : 0;
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < EM; ++j) {
        if (E_T || j < E) {
          const float d = vp[j] - xs[qc + j * tau];
          acc = acc + d * d;
        }
      }
      topk_offer<K>(qk, qi, acc, q, valid && abs(s - p0) > excl);
    };

    int s = -(kWave - 1);
#pragma unroll 1
    for (; s < 0; ++s) step_masked(s);  // head: low lanes still before q = 0
    if constexpr (T1 && E_T > 0) {
      const int s_full = m - (kWave - 1);  // steps s < s_full have every lane's q < m
      if (s + kUnroll <= s_full) {
        float win[E_T + kUnroll - 1];
#pragma unroll
        for (int j = 0; j < E_T - 1; ++j) win[j] = xs[s + lane + j];
        for (; s + kUnroll <= s_full; s += kUnroll) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) win[E_T - 1 + u] = xs[s + lane + E_T - 1 + u];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < E_T; ++j) {
              const float d = vp[j] - win[u + j];
              acc = acc + d * d;
            }
            topk_offer<K>(qk, qi, acc, s + u + lane, abs(s + u - p0) > excl);
          }
#pragma unroll
          for (int j = 0; j < E_T - 1; ++j) win[j] = win[j + kUnroll];
        }
      }
    }
#pragma unroll 1
    for (; s < m; ++s) step_masked(s);  // remainder and tail
  }

  // Epilogue: float64 distances of the k winners, weights, outputs.  The
  // loops over the winners stay rolled and rotate the register lists by one
  // slot per trip, so only one neighbour's coordinates are live at a time.
  Mom mine = mom_zero();
  if (active) {
    double D[K];  // distance, then weight, of neighbour qi[i]
    float Df[K];  // distance rounded for output
    double dmin = __builtin_inf();
#pragma unroll 1
    for (int r = 0; r < K; ++r) {
      // A slot stays unfilled (-1) only if non-finite input made keys NaN;
      // the status word reports that case, and index 0 keeps tables in range.
      const int q = qi[0] < 0 ? 0 : qi[0];
      double s2 = 0.0;
#pragma unroll
      for (int j = 0; j < EM; ++j) {
        if (E_T || j < E) {
          const double d = static_cast<double>(vp[j]) - static_cast<double>(xs[q + j * tau]);
          s2 += d * d;
        }
      }
      const double dq = sqrt(s2);
      dmin = fmin(dmin, dq);
#pragma unroll
      for (int i = 0; i < K - 1; ++i) {
        qi[i] = qi[i + 1];
        D[i] = D[i + 1];
        Df[i] = Df[i + 1];
      }
      qi[K - 1] = q;
      D[K - 1] = dq;
      Df[K - 1] = static_cast<float>(dq);
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
    const int64_t base = static_cast<int64_t>(slot) * a.tbl_stride + static_cast<int64_t>(p) * K;
    if (a.idx) {
#pragma unroll
      for (int i = 0; i < K; ++i) a.idx[base + i] = qi[i];
    }
    if (a.dist) {
#pragma unroll
      for (int i = 0; i < K; ++i) a.dist[base + i] = Df[i];
    }
    if (a.w) {
#pragma unroll
      for (int i = 0; i < K; ++i) a.w[base + i] = static_cast<float>(D[i] * inv);
    }
    if (a.mom) {
      const int o_off = off + a.Tp;
      double yh = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i) yh += (D[i] * inv) * static_cast<double>(xs[qi[i] + o_off]);
      mine.n = 1.0;
      mine.mo = static_cast<double>(xs[p + o_off]);
      mine.mp = yh;
    }
  }
  if (a.mom) {  // uniform
    const Mom wv = mom_wave_reduce(mine);
    if (lane == 0) wmom[threadIdx.x / kWave] = wv;
    __syncthreads();
    if (threadIdx.x == 0) {
      Mom t = wmom[0];
#pragma unroll
      for (int i = 1; i < kKnnThreads / kWave; ++i) t = mom_merge(t, wmom[i]);
      a.mom[(static_cast<int64_t>(row) * a.E_max + (E - 1)) * a.mom_blocks + blockIdx.x] = t;
    }
  }
}

template <int E_T, int K, bool T1>
hipError_t launch_one(const KnnArgs &a, dim3 grid, size_t shm, int slot0, hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_knn<E_T, K, T1>);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_knn<E_T, K, T1>), grid, dim3(kKnnThreads), shm, st, a, slot0);
  return hipGetLastError();
}

using LaunchFn = hipError_t (*)(const KnnArgs &, dim3, size_t, int, hipStream_t);

template <int E>
hipError_t launch_fast(const KnnArgs &a, dim3 grid, size_t shm, int slot0, hipStream_t st) {
  if (a.tau == 1) return launch_one<E, E + 1, true>(a, grid, shm, slot0, st);
  return launch_one<E, E + 1, false>(a, grid, shm, slot0, st);
}

template <int K>
hipError_t launch_generic(const KnnArgs &a, dim3 grid, size_t shm, int slot0, hipStream_t st) {
  return launch_one<0, K, false>(a, grid, shm, slot0, st);
}

template <size_t... I>
constexpr auto make_fast(std::index_sequence<I...>) {
  return std::array<LaunchFn, sizeof...(I)>{&launch_fast<static_cast<int>(I) + 1>...};
}
template <size_t... I>
constexpr auto make_generic(std::index_sequence<I...>) {
  return std::array<LaunchFn, sizeof...(I)>{&launch_generic<static_cast<int>(I) + 1>...};
}

}  // namespace

hipError_t launch_knn(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st) {
  static const auto fast = make_fast(std::make_index_sequence<EDM_E_MAX>{});
  static const auto generic = make_generic(std::make_index_sequence<EDM_K_MAX>{});
  if (nslots <= 0) return hipSuccess;
  const int64_t m_max = L_max;  // upper bound on queries per series
  const dim3 grid_x(static_cast<unsigned>((m_max + kKnnThreads - 1) / kKnnThreads));
  const size_t shm = static_cast<size_t>(L_max) * sizeof(float);
  LaunchFn fn = (a.k == a.E + 1 && a.E >= 1 && a.E <= EDM_E_MAX) ? fast[a.E - 1] : generic[a.k - 1];
  TimedLaunch timed(EDM_KF_EXACT_SCAN, st);
  constexpr int kMaxY = 32768;
  for (int s0 = 0; s0 < nslots; s0 += kMaxY) {
    const int ny = nslots - s0 < kMaxY ? nslots - s0 : kMaxY;
    hipError_t e = fn(a, dim3(grid_x.x, static_cast<unsigned>(ny)), shm, s0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace edm
