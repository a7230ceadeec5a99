// Small kernels: E-sweep epilogue, fill, and the stand-alone embedding.
#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

namespace edm {
namespace {

// One thread per series: merge the per-block co-moments of each E, write
// rho (NaN where E is infeasible or a side is constant) and pick the smallest
// E with the largest non-NaN rho (0 if none).  The selection is made on the
// float64 correlation before it is rounded for output.
__global__ void k_sweep_finalize(const Mom *__restrict__ mom, int32_t mom_blocks,
                                 const int64_t *__restrict__ L, int64_t N, int32_t E_max,
                                 int32_t tau, int32_t Tp, int32_t excl,
                                 const uint32_t *__restrict__ cand, float *__restrict__ rho,
                                 int32_t *__restrict__ E_opt) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= N) return;
  double best = -__builtin_inf();
  int best_e = 0;
  for (int E = 1; E <= E_max; ++E) {
    const int64_t m = L[s] - static_cast<int64_t>(E - 1) * tau - Tp;
    double r = __builtin_nan("");
    const bool evaluated = cand == nullptr || ((cand[s] >> (E - 1)) & 1u);
    if (evaluated && m - 1 - 2 * excl >= E + 1) {
      const int nb = static_cast<int>((m + kKnnThreads - 1) / kKnnThreads);
      const Mom *base = mom + (s * E_max + (E - 1)) * static_cast<int64_t>(mom_blocks);
      Mom t = base[0];
      for (int b = 1; b < nb; ++b) t = mom_merge(t, base[b]);
      r = mom_rho(t);
    }
    rho[s * E_max + (E - 1)] = static_cast<float>(r);
    if (r == r && r > best) {
      best = r;
      best_e = E;
    }
  }
  E_opt[s] = best_e;
}

// Candidate E set of each series from the network's logits: the m_top
// largest classes (ties to the smaller E), or every E when the largest
// softmax probability is below min_conf.  Bit E-1 of cand[s] marks E.
__global__ void k_candidates(const float *__restrict__ logits, int64_t N, int32_t E_max,
                             int32_t m_top, float min_conf, uint32_t *__restrict__ cand) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const float *z = logits + s * EDM_NET_CLASSES;
  float mx = z[0];
  for (int j = 1; j < EDM_NET_CLASSES; ++j) mx = fmaxf(mx, z[j]);
  float sum = 0.0f;
  for (int j = 0; j < EDM_NET_CLASSES; ++j) sum += expf(z[j] - mx);
  const uint32_t all = E_max >= 32 ? 0xffffffffu : ((1u << E_max) - 1u);
  if (1.0f / sum < min_conf) {
    cand[s] = all;
    return;
  }
  uint32_t m = 0;
  for (int r = 0; r < m_top; ++r) {
    int best = -1;
    for (int j = 0; j < EDM_NET_CLASSES; ++j)
      if (!((m >> j) & 1u) && (best < 0 || z[j] > z[best])) best = j;
    m |= 1u << best;
  }
  m &= all;
  cand[s] = m ? m : all;
}

// One workgroup of 1024 threads: histogram of E in LDS, exclusive scan,
// then a stable scatter in chunks of 1024 targets (per bin, each wave counts
// its lanes with a ballot; waves are ranked in order), so a bucket lists its
// targets in ascending order on every run.
constexpr int kGroupThreads = 1024;
constexpr int kBins = EDM_E_MAX + 1;
__global__ __launch_bounds__(kGroupThreads) void k_group_by_E(const int32_t *__restrict__ E, int64_t N,
                                                              int32_t E_max, int32_t *__restrict__ at,
                                                              int32_t *__restrict__ ids) {
  constexpr int kW = kGroupThreads / kWave;
  __shared__ int cnt[kBins];
  __shared__ int base[kBins];
  __shared__ int wc[kW][kBins];
  const int t = static_cast<int>(threadIdx.x);
  const int lane = t & (kWave - 1), wv = t / kWave;
  if (t < kBins) cnt[t] = 0;
  __syncthreads();
  auto bin = [&](int64_t j) {
    const int e = E[j];
    return (e >= 1 && e <= E_max) ? e : 0;
  };
  for (int64_t j = t; j < N; j += kGroupThreads) atomicAdd(&cnt[bin(j)], 1);
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int b = 0; b < kBins; ++b) {
      base[b] = acc;
      at[b] = acc;
      acc += cnt[b];
    }
    at[kBins] = acc;
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int64_t c0 = 0; c0 < N; c0 += kGroupThreads) {
    const int64_t j = c0 + t;
    const int b = j < N ? bin(j) : -1;
    int rank = 0;
    for (int q = 0; q < kBins; ++q) {
      const uint64_t m = __builtin_amdgcn_ballot_w64(b == q);
      if (b == q) rank = __builtin_popcountll(m & below);
      if (lane == 0) wc[wv][q] = __builtin_popcountll(m);
    }
    __syncthreads();
    if (b >= 0) {
      int off = base[b];
      for (int w = 0; w < wv; ++w) off += wc[w][b];
      ids[off + rank] = static_cast<int32_t>(j);
    }
    __syncthreads();
    if (t < kBins) {
      int add = 0;
      for (int w = 0; w < kW; ++w) add += wc[w][t];
      base[t] += add;
    }
    __syncthreads();
  }
}

__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t n, int64_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// out[p][j] = x[p + j*tau]; consecutive threads write consecutive elements.
// Row copy between a row subset of one array and a packed array:
// gather: dst[i] = src[ids[i]], scatter: dst[ids[i]] = src[i] (rows of
// `words` 32-bit words, leading dimensions in words).
__global__ void k_copy_rows(const uint32_t *__restrict__ src, int64_t lds, uint32_t *__restrict__ dst,
                            int64_t ldd, const int32_t *__restrict__ ids, int64_t words, int scatter) {
  const int64_t i = blockIdx.y;
  const int64_t r = ids[i];
  const uint32_t *s = src + (scatter ? i : r) * lds;
  uint32_t *d = dst + (scatter ? r : i) * ldd;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
       w += static_cast<int64_t>(gridDim.x) * blockDim.x)
    d[w] = s[w];
}

__global__ void k_embed(const float *__restrict__ x, int64_t n, int32_t E, int32_t tau,
                        float *__restrict__ out, int *status) {
  const int64_t total = n * E;
  bool bad = false;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t p = e / E;
    const int j = static_cast<int>(e - p * E);
    const float v = x[p + static_cast<int64_t>(j) * tau];
    bad |= !isfinite(v);
    out[e] = v;
  }
  if (bad) atomicOr(status, 1);
}

unsigned grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<unsigned>(b);
}

}  // namespace

hipError_t launch_sweep_finalize(const Mom *mom, int32_t mom_blocks, const int64_t *L_dev,
                                 int64_t N, int32_t E_max, int32_t tau, int32_t Tp, int32_t excl,
                                 const uint32_t *cand, float *rho, int32_t *E_opt,
                                 hipStream_t st) {
  if (N <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_FINALIZE, st);
  hipLaunchKernelGGL(k_sweep_finalize, dim3(grid_for(N, 64)), dim3(64), 0, st, mom, mom_blocks,
                     L_dev, N, E_max, tau, Tp, excl, cand, rho, E_opt);
  return hipGetLastError();
}

hipError_t launch_group_by_E(const int32_t *E, int64_t N, int32_t E_max, int32_t *at, int32_t *ids,
                             hipStream_t st) {
  if (N < 0 || N > INT32_MAX || E_max < 1 || E_max > EDM_E_MAX) return hipErrorInvalidValue;
  TimedLaunch timed(EDM_KF_GROUP, st);
  hipLaunchKernelGGL(k_group_by_E, dim3(1), dim3(kGroupThreads), 0, st, E, N, E_max, at, ids);
  return hipGetLastError();
}

hipError_t launch_candidates(const float *logits, int64_t N, int32_t E_max, int32_t m_top,
                             float min_conf, uint32_t *cand, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_OTHER, st);
  hipLaunchKernelGGL(k_candidates, dim3(grid_for(N, 64)), dim3(64), 0, st, logits, N, E_max,
                     m_top, min_conf, cand);
  return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_OTHER, st);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_OTHER, st);
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const void *src, int64_t lds, void *dst, int64_t ldd, const int32_t *ids,
                            int64_t n, int64_t words, bool scatter, hipStream_t st) {
  if (n <= 0 || words <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_OTHER, st);
  const int64_t wb = (words + 255) / 256;
  const unsigned gx = static_cast<unsigned>(wb < 64 ? wb : 64);
  constexpr int64_t kMaxY = 32768;
  for (int64_t c0 = 0; c0 < n; c0 += kMaxY) {  // packed side offset by c0 rows
    const int64_t nc = n - c0 < kMaxY ? n - c0 : kMaxY;
    const uint32_t *s = static_cast<const uint32_t *>(src) + (scatter ? c0 * lds : 0);
    uint32_t *d = static_cast<uint32_t *>(dst) + (scatter ? 0 : c0 * ldd);
    hipLaunchKernelGGL(k_copy_rows, dim3(gx, static_cast<unsigned>(nc)), dim3(256), 0, st, s, lds, d, ldd,
                       ids + c0, words, scatter ? 1 : 0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_embed(const float *x, int64_t L, int32_t E, int32_t tau, float *out,
                        int *status, hipStream_t st) {
  const int64_t n = L - static_cast<int64_t>(E - 1) * tau;
  TimedLaunch timed(EDM_KF_OTHER, st);
  hipLaunchKernelGGL(k_embed, dim3(grid_for(n * E, 256)), dim3(256), 0, st, x, n, E, tau, out,
                     status);
  return hipGetLastError();
}

}  // namespace edm
