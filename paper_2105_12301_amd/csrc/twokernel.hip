// The paper's two-kernel all-kNN (Section 3.3), kept as an ablation of the
// fused scans in knn.hip: Algorithm 1 writes the whole distance matrix of a
// library to device memory, then Algorithm 2 reads every row back and keeps
// its k smallest entries.  Results are identical to the fused form: the
// matrix holds the same float32 keys (lags ascending, one rounding per
// operation, no contraction), the selection is the same (key, index) order,
// and the epilogue repeats the fused kernel's float64 arithmetic in the same
// order, so tables, weights and the sweep's co-moments agree bit for bit.
//
// Design for gfx950
// -----------------
// * Distances (Algorithm 1): a workgroup owns 64 query rows x 256 candidate
//   columns of one library.  Each thread holds one candidate's E samples in
//   registers; the 64 queries' samples sit in LDS and are read as wave-wide
//   broadcasts; every row of the tile is one coalesced 1 KiB store.  For E = 1
//   the kernel moves 4 bytes per 3 ops and is bound by HBM writes, as the
//   paper found on its GPU.
// * Row top-k (Algorithm 2): the paper gives each row a team whose threads
//   keep private priority queues in scratch memory and merges them.  Here the
//   team is a wave: lane l reads the row in 16-byte pieces at columns
//   4l + 256c (coalesced), keeps a sorted register list of its k best
//   (key, q), and the 64 lists are merged by k rounds of a wave-wide
//   lexicographic minimum.  A workgroup's four waves do the 256 rows of one
//   query block and leave the winners in LDS; then each thread takes one
//   query of the block through the float64 epilogue, as the fused kernel
//   does, so the per-block co-moments are merged in the same order.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

#pragma clang fp contract(off)

namespace edm {
namespace {

constexpr int kDistCols = 256;  // candidates per distance workgroup (one per thread)
constexpr int kDistRows = 64;   // query rows per distance workgroup

template <int E_T>
__global__ __launch_bounds__(kDistCols) void k_distances(KnnArgs a, int slot0, float *__restrict__ D,
                                                         int64_t ldd) {
  __shared__ float vr[E_T][kDistRows];  // queries' samples, [lag][row]
  const int slot = slot0 + static_cast<int>(blockIdx.z);
  const int row = a.lib_ids ? a.lib_ids[slot] : slot;
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int tau = a.tau;
  const int m = L - (E_T - 1) * tau - a.Tp;
  const int p0 = static_cast<int>(blockIdx.y) * kDistRows;
  const int q = static_cast<int>(blockIdx.x) * kDistCols + static_cast<int>(threadIdx.x);
  if (m < 1 || p0 >= m || static_cast<int>(blockIdx.x) * kDistCols >= m) return;  // uniform

  bool bad = false;
  for (int i = threadIdx.x; i < E_T * kDistRows; i += kDistCols) {
    const int j = i / kDistRows, r = i % kDistRows;
    const int p = p0 + r;
    const float v = p < m ? x[p + j * tau] : 0.0f;
    bad |= !isfinite(v);
    vr[j][r] = v;
  }
  const bool valid = q < m;
  float vq[E_T];
#pragma unroll
  for (int j = 0; j < E_T; ++j) {
    vq[j] = valid ? x[q + j * tau] : 0.0f;
    bad |= !isfinite(vq[j]);
  }
  if (bad) atomicOr(a.status, 1);
  __syncthreads();

  float *__restrict__ out = D + static_cast<int64_t>(blockIdx.z) * ldd * ldd;
  const int rows = m - p0 < kDistRows ? m - p0 : kDistRows;
#pragma unroll 4
  for (int r = 0; r < rows; ++r) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < E_T; ++j) {
      const float d = vr[j][r] - vq[j];
      acc = acc + d * d;
    }
    if (valid) out[static_cast<int64_t>(p0 + r) * ldd + q] = acc;
  }
}

// Sorted insertion into an ascending register list (a lane's candidates come
// in ascending q, so strict comparisons keep equal keys in index order; a key
// not below the last entry leaves the list unchanged).
template <int K>
__device__ __forceinline__ void list_insert(float (&qk)[K], int (&qi)[K], float key, int q) {
#pragma unroll
  for (int i = K - 1; i > 0; --i) {
    const bool lt_prev = key < qk[i - 1];
    const bool lt_cur = key < qk[i];
    qi[i] = lt_prev ? qi[i - 1] : (lt_cur ? q : qi[i]);
    qk[i] = __builtin_amdgcn_fmed3f(qk[i - 1], key, qk[i]);
  }
  const bool lt0 = key < qk[0];
  qi[0] = lt0 ? q : qi[0];
  qk[0] = lt0 ? key : qk[0];
}

template <int K>
__device__ __forceinline__ void list_offer(float (&qk)[K], int (&qi)[K], float key, int q, bool ok) {
  const bool want = ok && key < qk[K - 1];
  if (__builtin_amdgcn_ballot_w64(want)) list_insert<K>(qk, qi, want ? key : __builtin_inff(), q);
}

template <int K>
__global__ __launch_bounds__(kKnnThreads) void k_row_topk(KnnArgs a, int slot0, const float *__restrict__ D,
                                                          int64_t ldd) {
  __shared__ int nbr[kKnnThreads * K];
  __shared__ Mom wmom[kKnnThreads / kWave];
  const int slot = slot0 + static_cast<int>(blockIdx.y);
  const int row = a.lib_ids ? a.lib_ids[slot] : slot;
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int E = a.E;
  const int tau = a.tau;
  const int off = (E - 1) * tau;
  const int m = L - off - a.Tp;
  const int excl = a.excl;  // exclusion radius: |q - p| <= excl is no candidate
  if (m - 1 - 2 * excl < K) return;  // infeasible for this series (uniform)
  const int blk0 = static_cast<int>(blockIdx.x) * kKnnThreads;
  if (blk0 >= m) return;

  const float *__restrict__ Dl = D + static_cast<int64_t>(blockIdx.y) * ldd * ldd;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;

  // Algorithm 2: the k smallest (key, q) of each of the wave's 64 rows.
#pragma unroll 1
  for (int r = 0; r < kWave; ++r) {
    const int p = blk0 + wv * kWave + r;
    if (p >= m) break;  // wave-uniform
    const float *__restrict__ Dr = Dl + static_cast<int64_t>(p) * ldd;
    float qk[K];
    int qi[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      qk[i] = __builtin_inff();
      qi[i] = -1;
    }
    for (int c = 4 * lane; c - 4 * lane < m; c += 4 * kWave) {
      // ldd is a multiple of 64, so the 16-byte piece stays inside the row.
      const float4 v = c < m ? *reinterpret_cast<const float4 *>(Dr + c) : float4{0, 0, 0, 0};
      list_offer<K>(qk, qi, v.x, c + 0, c + 0 < m && abs(c + 0 - p) > excl);
      list_offer<K>(qk, qi, v.y, c + 1, c + 1 < m && abs(c + 1 - p) > excl);
      list_offer<K>(qk, qi, v.z, c + 2, c + 2 < m && abs(c + 2 - p) > excl);
      list_offer<K>(qk, qi, v.w, c + 3, c + 3 < m && abs(c + 3 - p) > excl);
    }
    // Merge the 64 lane lists: k rounds of a lexicographic wave minimum; the
    // winning lane drops its head.  Indices are distinct across lanes, so one
    // lane wins (unfilled entries (inf, -1) only tie with each other).
#pragma unroll 1
    for (int t = 0; t < K; ++t) {
      float bk = qk[0];
      int bq = qi[0];
#pragma unroll
      for (int s = 1; s < kWave; s <<= 1) {
        const float ok = __shfl_xor(bk, s);
        const int oq = __shfl_xor(bq, s);
        const bool take = ok < bk || (ok == bk && oq < bq);
        bk = take ? ok : bk;
        bq = take ? oq : bq;
      }
      if (qk[0] == bk && qi[0] == bq) {
#pragma unroll
        for (int i = 0; i < K - 1; ++i) {
          qk[i] = qk[i + 1];
          qi[i] = qi[i + 1];
        }
        qk[K - 1] = __builtin_inff();
        qi[K - 1] = -1;
      }
      if (lane == 0) nbr[(wv * kWave + r) * K + t] = bq;
    }
  }
  __syncthreads();

  // Epilogue, one query per thread: the fused kernel's float64 arithmetic in
  // the same order (distances of the k winners, d_min, weights, outputs).
  const int p = blk0 + static_cast<int>(threadIdx.x);
  const bool active = p < m;
  Mom mine = mom_zero();
  if (active) {
    float vp[EDM_E_MAX];
#pragma unroll
    for (int j = 0; j < EDM_E_MAX; ++j) vp[j] = j < E ? x[p + j * tau] : 0.0f;
    int qi[K];
#pragma unroll
    for (int i = 0; i < K; ++i) qi[i] = nbr[threadIdx.x * K + i];
    double D2[K];
    float Df[K];
    double dmin = __builtin_inf();
#pragma unroll 1
    for (int r = 0; r < K; ++r) {
      const int q = qi[0] < 0 ? 0 : qi[0];
      double s2 = 0.0;
#pragma unroll
      for (int j = 0; j < EDM_E_MAX; ++j) {
        if (j < E) {
          const double d = static_cast<double>(vp[j]) - static_cast<double>(x[q + j * tau]);
          s2 += d * d;
        }
      }
      const double dq = sqrt(s2);
      dmin = fmin(dmin, dq);
#pragma unroll
      for (int i = 0; i < K - 1; ++i) {
        qi[i] = qi[i + 1];
        D2[i] = D2[i + 1];
        Df[i] = Df[i + 1];
      }
      qi[K - 1] = q;
      D2[K - 1] = dq;
      Df[K - 1] = static_cast<float>(dq);
    }
    double wsum = 0.0;
#pragma unroll 1
    for (int r = 0; r < K; ++r) {
      const double d = D2[0];
      const double wq = dmin > 0.0 ? exp(-d / dmin) : (d == 0.0 ? 1.0 : 0.0);
      wsum += wq;
#pragma unroll
      for (int i = 0; i < K - 1; ++i) D2[i] = D2[i + 1];
      D2[K - 1] = wq;
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
      for (int i = 0; i < K; ++i) a.w[base + i] = static_cast<float>(D2[i] * inv);
    }
    if (a.mom) {
      const int o_off = off + a.Tp;
      double yh = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i) yh += (D2[i] * inv) * static_cast<double>(x[qi[i] + o_off]);
      mine.n = 1.0;
      mine.mo = static_cast<double>(x[p + o_off]);
      mine.mp = yh;
    }
  }
  if (a.mom) {  // uniform
    const Mom wm = mom_wave_reduce(mine);
    if (lane == 0) wmom[wv] = wm;
    __syncthreads();
    if (threadIdx.x == 0) {
      Mom t = wmom[0];
#pragma unroll
      for (int i = 1; i < kKnnThreads / kWave; ++i) t = mom_merge(t, wmom[i]);
      a.mom[(static_cast<int64_t>(row) * a.E_max + (E - 1)) * a.mom_blocks + blockIdx.x] = t;
    }
  }
}

using DistFn = void (*)(KnnArgs, int, float *, int64_t);
using TopkFn = void (*)(KnnArgs, int, const float *, int64_t);

template <size_t... I>
constexpr auto make_dist(std::index_sequence<I...>) {
  return std::array<DistFn, sizeof...(I)>{&k_distances<static_cast<int>(I) + 1>...};
}
template <size_t... I>
constexpr auto make_topk(std::index_sequence<I...>) {
  return std::array<TopkFn, sizeof...(I)>{&k_row_topk<static_cast<int>(I) + 1>...};
}

}  // namespace

int64_t two_kernel_ld(int64_t m_max) { return (m_max + 63) / 64 * 64; }

hipError_t launch_knn_two_kernel(const KnnArgs &a, int nslots, int64_t L_max, float *D, int64_t ldd,
                                 int slots_per_pass, hipStream_t st) {
  static const auto dist = make_dist(std::make_index_sequence<EDM_E_MAX>{});
  static const auto topk = make_topk(std::make_index_sequence<EDM_K_MAX>{});
  if (nslots <= 0) return hipSuccess;
  if (a.E < 1 || a.E > EDM_E_MAX || a.k < 1 || a.k > EDM_K_MAX || slots_per_pass < 1) return hipErrorInvalidValue;
  const int64_t m_max = L_max - static_cast<int64_t>(a.E - 1) * a.tau - a.Tp;
  if (m_max < 1) return hipSuccess;
  if (ldd < m_max || ldd % 64 != 0) return hipErrorInvalidValue;
  const unsigned col_tiles = static_cast<unsigned>((m_max + kDistCols - 1) / kDistCols);
  const unsigned row_tiles = static_cast<unsigned>((m_max + kDistRows - 1) / kDistRows);
  const unsigned qblocks = static_cast<unsigned>((m_max + kKnnThreads - 1) / kKnnThreads);
  constexpr int kMaxZ = 65535;
  for (int s0 = 0; s0 < nslots; s0 += slots_per_pass) {
    const int nb0 = nslots - s0 < slots_per_pass ? nslots - s0 : slots_per_pass;
    {
      TimedLaunch timed(EDM_KF_DISTANCES, st);
      for (int z0 = 0; z0 < nb0; z0 += kMaxZ) {
        const int nz = nb0 - z0 < kMaxZ ? nb0 - z0 : kMaxZ;
        hipLaunchKernelGGL(dist[a.E - 1], dim3(col_tiles, row_tiles, static_cast<unsigned>(nz)),
                           dim3(kDistCols), 0, st, a, s0 + z0, D + static_cast<int64_t>(z0) * ldd * ldd, ldd);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    {
      TimedLaunch timed(EDM_KF_ROW_TOPK, st);
      for (int y0 = 0; y0 < nb0; y0 += kMaxZ) {
        const int ny = nb0 - y0 < kMaxZ ? nb0 - y0 : kMaxZ;
        hipLaunchKernelGGL(topk[a.k - 1], dim3(qblocks, static_cast<unsigned>(ny)), dim3(kKnnThreads), 0,
                           st, a, s0 + y0, D + static_cast<int64_t>(y0) * ldd * ldd, ldd);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipSuccess;
}

}  // namespace edm
