// Cross-map tables from the E sweep's neighbour lists (kEDM paper: Section
// 3.4 runs the simplex E sweep and then the cross map of every pair at the
// target's E; both need every library's k-nearest-neighbour table at that E).
//
// The sweep predicts Tp = 1 ahead: at dimension E (tau = 1) its queries and
// candidates are the m1 = L - E first embedded points.  The cross map at
// Tp = 0 has m0 = m1 + 1 of each: one more candidate, index m1, and one more
// query, p = m1.  For p < m1 the Tp = 0 list is therefore the sweep's list
// with candidate m1 offered last; it has the largest index, so a strict "<"
// puts it after equal keys, exactly where a full scan would (and where it
// does not enter, the sweep's weights are the table's).  Query p = m1 is
// scanned in full.  A series with no sweep list at E (m1 - 1 < E + 1) but
// a defined cross map (m0 - 1 >= E + 1) has every query scanned.
// Keys are the float32 sums of Algorithm 1 (contraction off), so the tables
// are bit-identical to the scans'.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"
#include "scan_common.h"

#pragma clang fp contract(off)

namespace edm {
namespace {

template <int E>
__device__ __forceinline__ float canon_key(const float *__restrict__ xs, int p, int q) {
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const float d = xs[p + j] - xs[q + j];
    acc = acc + d * d;
  }
  return acc;
}

__device__ __forceinline__ void stage(const KnnArgs &a, int row, int L, float *xs) {
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  for (int i = threadIdx.x; i < L; i += blockDim.x) xs[i] = x[i];
  __syncthreads();
}

// Queries p < m1: one thread per query, the series read from global memory
// (L2).  The sweep's list is the cross map's unless candidate m1 enters it,
// that is unless key(p, m1) < key(p, last entry); then the list and the
// weights the sweep kept are the table row (the weights depend only on the
// query and its neighbours), and when the table is the kept array itself the
// row is left as it is.  Otherwise (about one query in a hundred) the query
// is queued in LDS, and the queue is worked off by consecutive threads: every
// key is recomputed, m1 is inserted and the row is rewritten (the kept
// entries are read before).
template <int E>
__global__ __launch_bounds__(256) void k_fix_from_sweep(KnnArgs a, int slot0) {
  constexpr int K = E + 1;
  if (a.group_at && a.group_at[E + 1] == a.group_at[E]) return;  // no target of this E
  const int row = slot0 + static_cast<int>(blockIdx.y);
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int m1 = L - E;
  if (m1 - 1 < K) return;  // no sweep list: k_scan_queries covers this series
  if (static_cast<int>(blockIdx.x) * 256 >= m1) return;  // (uniform)
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  auto key_of = [&](int p, int q) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const float d = x[p + j] - x[q + j];
      acc = acc + d * d;
    }
    return acc;
  };
  // Queries where m1 enters the list (about 1 in 100) are queued in LDS and
  // rewritten by consecutive threads, so the slow path runs on few waves.
  __shared__ int queue[256];
  __shared__ int n_queue;
  if (threadIdx.x == 0) n_queue = 0;
  __syncthreads();
  const int p = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  const bool same = a.idxE[E] == a.keepE[E] && a.wE[E] == a.keepWE[E] && a.strideE[E] == a.keep_strideE[E];
  if (p < m1) {
    const int64_t ko = static_cast<int64_t>(row) * a.keep_strideE[E] + static_cast<int64_t>(p) * K;
    const int32_t *__restrict__ kp = a.keepE[E] + ko;
    if (a.keepWE[E] && !(key_of(p, m1) < key_of(p, kp[K - 1]))) {
      // the kept row is the table row: nothing to do when the table is the
      // kept array itself (one extra row per slot for query m1), else a copy
      if (!same) {
        const int64_t base = static_cast<int64_t>(row) * a.strideE[E] + static_cast<int64_t>(p) * K;
        const float *__restrict__ kw = a.keepWE[E] + ko;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          a.idxE[E][base + i] = kp[i];
          a.wE[E][base + i] = kw[i];
        }
      }
    } else {
      queue[atomicAdd(&n_queue, 1)] = p;
    }
  }
  __syncthreads();
  const int nq = n_queue;
  for (int i = static_cast<int>(threadIdx.x); i < nq; i += 256) {
    const int pq = queue[i];
    const int32_t *__restrict__ kp =
        a.keepE[E] + static_cast<int64_t>(row) * a.keep_strideE[E] + static_cast<int64_t>(pq) * K;
    float vp[E];
#pragma unroll
    for (int j = 0; j < E; ++j) vp[j] = x[pq + j];
    const float k_m1 = key_of(pq, m1);
    // m1 enters after every entry whose key is at most its own (it has the
    // largest index) and pushes the last entry out.
    int pos = 0;
#pragma unroll 1
    for (int r = 0; r < K; ++r) pos += key_of(pq, kp[r]) <= k_m1 ? 1 : 0;
    int qi[K];
#pragma unroll
    for (int r = 0; r < K; ++r) qi[r] = r < pos ? kp[r] : (r == pos ? m1 : kp[r - 1 < 0 ? 0 : r - 1]);
    finish_list<E, 0, K, E>(a, row, pq, L, 0, a.need, vp, qi, x);
  }
}

// Full scans, one query per wave: the lanes walk the candidates in ascending
// order keeping their own sorted lists, then the K smallest (key, index) of
// the 64 lists are taken one at a time (lexicographic, ties to the lower
// index).  Query m1 of every series, or every query of a series whose sweep
// had no list at E.
template <int E>
__global__ __launch_bounds__(256) void k_scan_queries(KnnArgs a, int slot0) {
  constexpr int K = E + 1;
  extern __shared__ float fx_xs[];
  if (a.group_at && a.group_at[E + 1] == a.group_at[E]) return;  // no target of this E
  const int row = slot0 + static_cast<int>(blockIdx.y);
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int m0 = L - (E - 1), m1 = m0 - 1;
  if (m0 - 1 < K) return;  // the cross map is undefined at E for this library
  stage(a, row, L, fx_xs);
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  const int lane = static_cast<int>(threadIdx.x) & (kWave - 1);
  const int p_first = (m1 - 1 < K) ? 0 : m1;
  for (int p = p_first + wave; p < m0; p += static_cast<int>(blockDim.x) / kWave) {
    float qk[K];
    int qi[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      qk[i] = __builtin_inff();
      qi[i] = -1;
    }
    for (int q = lane; q < m0; q += kWave) {
      const float kq = q == p ? __builtin_inff() : canon_key<E>(fx_xs, p, q);
      if (kq < qk[K - 1]) slice_insert<0, K, K>(qk, qi, kq, q);
    }
    int ri[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
      float bk = qk[0];
      int bi = qi[0];
#pragma unroll
      for (int m = 1; m < kWave; m <<= 1) {
        const float ok = __shfl_xor(bk, m);
        const int oi = __shfl_xor(bi, m);
        if (ok < bk || (ok == bk && static_cast<uint32_t>(oi) < static_cast<uint32_t>(bi))) {
          bk = ok;
          bi = oi;
        }
      }
      ri[r] = bi;
      if (bi >= 0 && qi[0] == bi) {  // this lane held the winner: drop it
#pragma unroll
        for (int i = 0; i < K - 1; ++i) {
          qk[i] = qk[i + 1];
          qi[i] = qi[i + 1];
        }
        qk[K - 1] = __builtin_inff();
        qi[K - 1] = -1;
      }
    }
    if (lane == 0) {
      float vp[E];
#pragma unroll
      for (int j = 0; j < E; ++j) vp[j] = fx_xs[p + j];
      finish_list<E, 0, K, E>(a, row, p, L, 0, a.need, vp, ri, fx_xs);
    }
  }
}

using FixFn = hipError_t (*)(const KnnArgs &, int, int64_t, hipStream_t);

template <int E>
hipError_t launch_fix(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st) {
  const size_t shm = static_cast<size_t>(L_max) * sizeof(float);
  const void *f2 = reinterpret_cast<const void *>(&k_scan_queries<E>);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(f2, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  const unsigned gx = static_cast<unsigned>((L_max + 255) / 256);
  constexpr int kMaxY = 32768;
  for (int s0 = 0; s0 < nslots; s0 += kMaxY) {
    const unsigned ny = static_cast<unsigned>(nslots - s0 < kMaxY ? nslots - s0 : kMaxY);
    hipLaunchKernelGGL(k_fix_from_sweep<E>, dim3(gx, ny), dim3(256), 0, st, a, s0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_queries<E>, dim3(1, ny), dim3(256), shm, st, a, s0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <size_t... I>
constexpr std::array<FixFn, EDM_E_MAX> fix_table(std::index_sequence<I...>) {
  return {{&launch_fix<static_cast<int>(I) + 1>...}};
}

}  // namespace

hipError_t launch_tables_from_sweep(const KnnArgs &a, int E, int nslots, int64_t L_max,
                                    hipStream_t st) {
  static const std::array<FixFn, EDM_E_MAX> t = fix_table(std::make_index_sequence<EDM_E_MAX>{});
  if (E < 1 || E > EDM_E_MAX || a.tau != 1 || a.mom != nullptr || !a.keepE[E] || !a.idxE[E] ||
      !a.wE[E])
    return hipErrorInvalidValue;
  if (nslots <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_TABLES_FROM_SWEEP, st);
  return t[E - 1](a, nslots, L_max, st);
}

}  // namespace edm
