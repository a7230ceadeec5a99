// Neighbour tables on library subsamples, for the convergence test of CCM:
// the cross-map skill should grow with the library size when the target
// drives the library (the convergence criterion behind Section 2.1's method;
// the paper itself runs every pair on the whole series).  A subsample is a
// set of candidate points of the library; every query point p of the whole
// series takes its k nearest neighbours inside the set (p itself and its
// exclusion window barred), and the lookup and correlation then run over all
// query points as for the full library.
//
// Design for gfx950
// -----------------
// * One workgroup = 256 consecutive queries (one per lane) x one subsample.
//   The series sits in LDS, and the subsample's member indices are staged in
//   LDS chunks of kChunk; every lane walks the members in ascending order, so
//   a member's samples are one wave-wide broadcast LDS read per lag and the
//   work is O(queries x members x E) instead of a scan of every point.
// * The key is the float32 sum of Algorithm 1 (lags ascending, one rounding
//   per operation, this file compiled without contraction), the register
//   list and its ballot-gated insertion are the fused scan's, and the
//   float64 epilogue follows the same order, so a subsample holding every
//   point gives the fused scan's table bit for bit.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

#pragma clang fp contract(off)

namespace edm {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 4096;  // member indices staged per LDS chunk

template <int K>
__device__ __forceinline__ void sub_insert(float (&qk)[K], int (&qi)[K], float key, int q) {
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

// a.X / a.L_uni: the library series; a.idx / a.w: tables [set][m][K]
// (stride a.tbl_stride); members of set s: sets[off[s] .. off[s+1]).
template <int E_T, int K>
__global__ __launch_bounds__(kThreads) void k_knn_subset(KnnArgs a, const int32_t *__restrict__ sets,
                                                         const int64_t *__restrict__ off) {
  extern __shared__ float sub_smem[];
  const int E = E_T;
  const int tau = a.tau;
  const int L = static_cast<int>(a.L_uni);
  const int m = L - (E - 1) * tau - a.Tp;
  const int excl = a.excl;
  const int set = static_cast<int>(blockIdx.y);
  const int blk0 = static_cast<int>(blockIdx.x) * kThreads;
  if (blk0 >= m) return;
  float *xs = sub_smem;
  int32_t *mem = reinterpret_cast<int32_t *>(sub_smem + L);
  const float *__restrict__ x = a.X;
  bool bad = false;
  for (int i = threadIdx.x; i < L; i += kThreads) {
    const float v = x[i];
    bad |= !isfinite(v);
    xs[i] = v;
  }
  if (bad) atomicOr(a.status, 1);

  const int p = blk0 + static_cast<int>(threadIdx.x);
  const bool active = p < m;
  float vp[E_T];
#pragma unroll
  for (int j = 0; j < E_T; ++j) vp[j] = 0.0f;
  float qk[K];
  int qi[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    qk[i] = active ? __builtin_inff() : -1.0f;  // -1: an idle lane never inserts
    qi[i] = -1;
  }
  const int64_t b0 = off[set], b1 = off[set + 1];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < E_T; ++j) vp[j] = active ? xs[p + j * tau] : 0.0f;
  for (int64_t c0 = b0; c0 < b1; c0 += kChunk) {
    const int n = static_cast<int>(b1 - c0 < kChunk ? b1 - c0 : kChunk);
    __syncthreads();  // the previous chunk is consumed
    for (int i = threadIdx.x; i < n; i += kThreads) mem[i] = sets[c0 + i];
    __syncthreads();
#pragma unroll 2
    for (int i = 0; i < n; ++i) {
      const int q = mem[i];  // wave-uniform
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < E_T; ++j) {
        const float d = vp[j] - xs[q + j * tau];
        acc = acc + d * d;
      }
      const bool want = abs(q - p) > excl && acc < qk[K - 1];
      if (__builtin_amdgcn_ballot_w64(want)) sub_insert<K>(qk, qi, want ? acc : __builtin_inff(), q);
    }
  }
  if (!active) return;

  // Epilogue: float64 distances of the K winners, d_min, weights (Section
  // 2.1 step 3), in the fused scan's order.
  double D[K];
  double dmin = __builtin_inf();
#pragma unroll 1
  for (int r = 0; r < K; ++r) {
    const int q = qi[0] < 0 ? 0 : qi[0];
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < E_T; ++j) {
      const double d = static_cast<double>(vp[j]) - static_cast<double>(xs[q + j * tau]);
      s2 += d * d;
    }
    const double dq = sqrt(s2);
    dmin = fmin(dmin, dq);
#pragma unroll
    for (int i = 0; i < K - 1; ++i) {
      qi[i] = qi[i + 1];
      D[i] = D[i + 1];
    }
    qi[K - 1] = q;
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
  const int64_t base = static_cast<int64_t>(set) * a.tbl_stride + static_cast<int64_t>(p) * K;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    a.idx[base + i] = qi[i];
    a.w[base + i] = static_cast<float>(D[i] * inv);
  }
}

using SubFn = void (*)(KnnArgs, const int32_t *, const int64_t *);

template <size_t... I>
constexpr auto make_sub(std::index_sequence<I...>) {
  return std::array<SubFn, sizeof...(I)>{&k_knn_subset<static_cast<int>(I) + 1, static_cast<int>(I) + 2>...};
}

}  // namespace

hipError_t launch_knn_subsets(const KnnArgs &a, const int32_t *sets, const int64_t *off, int n_sets,
                              hipStream_t st) {
  static const auto fns = make_sub(std::make_index_sequence<EDM_E_MAX>{});
  if (n_sets <= 0) return hipSuccess;
  if (a.E < 1 || a.E > EDM_E_MAX || a.k != a.E + 1 || a.L_uni < 1 || a.L_uni > EDM_L_MAX ||
      !a.idx || !a.w)
    return hipErrorInvalidValue;
  const int64_t m = a.L_uni - static_cast<int64_t>(a.E - 1) * a.tau - a.Tp;
  if (m < 1) return hipSuccess;
  const size_t shm = static_cast<size_t>(a.L_uni) * sizeof(float) + kChunk * sizeof(int32_t);
  const void *fn = reinterpret_cast<const void *>(fns[a.E - 1]);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  TimedLaunch timed(EDM_KF_EXACT_SCAN, st);
  constexpr int kMaxY = 32768;
  const unsigned gx = static_cast<unsigned>((m + kThreads - 1) / kThreads);
  for (int s0 = 0; s0 < n_sets; s0 += kMaxY) {
    const int ny = n_sets - s0 < kMaxY ? n_sets - s0 : kMaxY;
    KnnArgs b = a;
    b.idx = a.idx + static_cast<int64_t>(s0) * a.tbl_stride;
    b.w = a.w + static_cast<int64_t>(s0) * a.tbl_stride;
    hipLaunchKernelGGL(fns[a.E - 1], dim3(gx, static_cast<unsigned>(ny)), dim3(kThreads), shm, st, b,
                       sets, off + s0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace edm
