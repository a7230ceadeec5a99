// Batched simplex lookup with the Pearson skill computed on the fly
// (kEDM paper: Section 2.1 steps 3-4, Section 3.4 and Algorithm 3).
//
// Data layout.  A workgroup stages a tile of T targets (T in 1, 2, 4, 8, 16,
// as many as fit 160 KB of LDS for the window) over the window that its
// libraries' tables can touch, interleaved: vs[e][t] = y_t[off + e] - c_t with
// c_t the target's mean (k_target_means, one value per target and call, the
// same for every kernel), off = (E-1)*tau + Tp, rows S = tile_stride(T) floats
// apart.
// One neighbour index q then addresses the T targets' samples as one
// contiguous LDS segment, so a wave reads them with one 128-, 64- or 32-bit
// access per lane instead of T scattered 32-bit gathers.  (Rows padded to
// T + 4 floats, which spreads the random rows over more bank offsets, made
// the headline lookups 5 % slower on gfx950; the rows are unpadded.)
//
// Lane layout.  A wave walks one library's table: lane = 4 g + s, query group
// g = 0..15 handles the queries p = g, g + 16, g + 32, ... and sub-lane s the
// targets s*TPL .. s*TPL + TPL - 1 of the tile (TPL = T/4 targets per lane, at
// least 1; for T < 4 some sub-lanes idle).  Per query the lane reads the table
// row (K indices and weights, shared by the 4 lanes of the group), gathers
// vs[q_i][targets] for i = 0..K-1 and accumulates the prediction
// yhat = sum_i w_i (y(t(q_i)+Tp) - c) with one float32 fused multiply-add per
// neighbour in index order, and the sums of the observation o = vs[p] and
// yhat: so, sp, soo, spp, sop, accumulated in float32 over runs of kRun
// queries and added to float64 totals after each run.  Both sides are taken
// relative to the target's mean (the weights sum to one, so the prediction's
// mean is near it too): the float32 runs then round values of the target's
// spread, not of its offset, and the correlation keeps errors of order 1e-8.
//
// Every pair's arithmetic is fixed: per query group the runs and the float64
// sums go over p in increasing order, then the 16 group sums meet in a
// butterfly over the lane bits of g (masks 4, 8, 16, 32).  It does not depend on T, on which
// kernel ran the pair or on how many libraries or targets shared a
// workgroup, so every kernel here and every form of the library give
// bit-identical rho.
//
// Grid kernel: blockIdx.x = tile of targets, blockIdx.y = group of 16
// library slots (one wave each); consecutive workgroups share their
// libraries' tables in L2.  Work-list kernel (batched plan): one item = a
// group of up to 16 libraries of similar length (longest first) against one
// tile, workgroups persistent or one per item.
#include <array>
#include <utility>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"

namespace edm {
namespace {

constexpr int kGroups = 16;                  // query groups per wave
constexpr int kRun = 8;                      // queries per float32 run of the skill sums
constexpr int kXcds = 8;                     // accelerator dies (separate L2 caches) of the chip
constexpr int kTileCols = 16;                // tile columns per library group (device buckets)
constexpr int kSubs = 4;                     // lanes per query group
constexpr int kWaves = kLookupItemLibs;      // libraries per workgroup, one wave each
constexpr int kThreads = kWaves * kWave;     // 1024
// staged targets: 160 KiB less 512 bytes for the kernels' static LDS (target
// ids, offsets, the item index)
constexpr int64_t kLdsFloats = (160 * 1024 - 512) / 4;

static_assert(kGroups * kSubs == kWave, "lane layout");
static_assert(kLookupItemMaxTargets == 16, "tile layout assumes at most 16 targets");

struct Sums {
  double so, sp, soo, spp, sop;
};

// Row stride (floats) of a staged tile of T targets.
__host__ __device__ constexpr int tile_stride(int T) { return T; }

template <int N>
struct VecOf;
template <>
struct VecOf<1> {
  using type = float;
};
template <>
struct VecOf<2> {
  using type = float2;
};
template <>
struct VecOf<4> {
  using type = float4;
};

template <int TPL>
__device__ __forceinline__ void lds_read(const float *p, float (&v)[TPL]) {
  using V = typename VecOf<TPL>::type;
  const V x = *reinterpret_cast<const V *>(p);
  if constexpr (TPL == 1) {
    v[0] = x;
  } else if constexpr (TPL == 2) {
    v[0] = x.x;
    v[1] = x.y;
  } else {
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
  }
}

// Skill sums of one wave's library against the staged tile (row stride T
// floats).  Lane (g, s) handles targets s*TPL + u of the tile; every lane
// returns the wave totals of its targets.  pred[u] (or null): prediction row
// of target u of the lane, written as yhat + c[u].
template <int K, int TPL, bool kPred>
__device__ __forceinline__ void tile_pairs(const int32_t *__restrict__ tidx,
                                           const float *__restrict__ tw, const int m,
                                           const float *vs, const int T, const int S,
                                           float *const (&pred)[TPL], const float (&c)[TPL],
                                           Sums (&s)[TPL]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane >> 2;
  const int sub = lane & (kSubs - 1);
  // idle sub-lanes (T < 4) read sub-lane 0's targets; their sums are unused
  const int col = sub * TPL < T ? sub * TPL : 0;
  const float *base = vs + col;
#pragma unroll
  for (int u = 0; u < TPL; ++u) s[u] = Sums{0.0, 0.0, 0.0, 0.0, 0.0};
  for (int p0 = g; p0 < m; p0 += kGroups * kRun) {
    const int pe = m < p0 + kGroups * kRun ? m : p0 + kGroups * kRun;
    float f[TPL][5];
#pragma unroll
    for (int u = 0; u < TPL; ++u)
#pragma unroll
      for (int j = 0; j < 5; ++j) f[u][j] = 0.0f;
    for (int p = p0; p < pe; p += kGroups) {
      const int64_t row = static_cast<int64_t>(p) * K;
      int q[K];
      float w[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        q[i] = tidx[row + i];
        w[i] = tw[row + i];
      }
      float yh[TPL];
#pragma unroll
      for (int u = 0; u < TPL; ++u) yh[u] = 0.0f;
      // gathers in chunks of kChunk neighbours (bounds the registers in flight)
      constexpr int kChunk = TPL == 4 ? 4 : (TPL == 2 ? 8 : 16);
#pragma unroll
      for (int i0 = 0; i0 < K; i0 += kChunk) {
        float v[kChunk][TPL];
        // The chunk's gathers are issued at a raised wave priority, so the
        // SIMD's waves keep the LDS queue fed before their arithmetic (the
        // lookups are bound by LDS throughput; 3 % faster on the
        // 10000 x 2000 step, results unchanged).
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int i = i0; i < (i0 + kChunk < K ? i0 + kChunk : K); ++i)
          lds_read<TPL>(base + __umul24(q[i], S), v[i - i0]);  // q < 2^24: one full-rate multiply
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int i = i0; i < (i0 + kChunk < K ? i0 + kChunk : K); ++i)
#pragma unroll
          for (int u = 0; u < TPL; ++u) yh[u] = fmaf(w[i], v[i - i0][u], yh[u]);
        if (K > kChunk) __builtin_amdgcn_sched_barrier(0);
      }
      float ov[TPL];
      lds_read<TPL>(base + __umul24(p, S), ov);
#pragma unroll
      for (int u = 0; u < TPL; ++u) {
        // explicit fused forms: the same operations in every instantiation
        f[u][0] += ov[u];
        f[u][1] += yh[u];
        f[u][2] = fmaf(ov[u], ov[u], f[u][2]);
        f[u][3] = fmaf(yh[u], yh[u], f[u][3]);
        f[u][4] = fmaf(ov[u], yh[u], f[u][4]);
        if constexpr (kPred) {
          if (pred[u]) pred[u][p] = yh[u] + c[u];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
      s[u].so += static_cast<double>(f[u][0]);
      s[u].sp += static_cast<double>(f[u][1]);
      s[u].soo += static_cast<double>(f[u][2]);
      s[u].spp += static_cast<double>(f[u][3]);
      s[u].sop += static_cast<double>(f[u][4]);
    }
  }
#pragma unroll
  for (int u = 0; u < TPL; ++u) {
#pragma unroll
    for (int msk = kSubs; msk < kWave; msk <<= 1) {
      s[u].so += __shfl_xor(s[u].so, msk);
      s[u].sp += __shfl_xor(s[u].sp, msk);
      s[u].soo += __shfl_xor(s[u].soo, msk);
      s[u].spp += __shfl_xor(s[u].spp, msk);
      s[u].sop += __shfl_xor(s[u].sop, msk);
    }
  }
}

__device__ __forceinline__ float pair_rho(int m, const Sums &s) {
  return static_cast<float>(
      mom_rho(mom_from_shifted_sums(static_cast<double>(m), 0.0, 0.0, s.so, s.sp, s.soo, s.spp, s.sop)));
}

// Stage targets tgt[0..Tn) over the window [off, off + n) into vs[e][t]
// (row stride S = tile_stride(T), targets Tn..T-1 zero), relative to
// cs[t] = a.cmean[target]; zero past a target's own length.  Ends with a
// barrier.
__device__ __forceinline__ void stage_tile(const LookupArgs &a, const int *tgt, int Tn, int T,
                                           int lgT, int off, int n, float *vs, float *cs) {
  const int S = tile_stride(T);
  if (static_cast<int>(threadIdx.x) < T) {
    const int t = threadIdx.x;
    cs[t] = t < Tn ? a.cmean[tgt[t]] : 0.0f;
  }
  __syncthreads();
  bool bad = false;
  const int total = n * T;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int e = idx >> lgT;
    const int t = idx & (T - 1);
    float v = 0.0f;
    if (t < Tn) {
      const int64_t Ly = a.Ly_dev ? a.Ly_dev[tgt[t]] : a.ldy;
      if (off + e < Ly) {
        const float y = a.Y[static_cast<int64_t>(tgt[t]) * a.ldy + off + e];
        bad |= !isfinite(y);
        v = y - cs[t];
      }
    }
    vs[e * S + t] = v;
  }
  if (bad) atomicOr(a.status, 1);
  __syncthreads();
}

// One wave's library (m queries, table tidx/tw) against the staged tile
// tgt[0..Tn): sums, then rho (and predictions) for the pairs that are
// defined (target at least as long as the library).
template <int K, int TPL>
__device__ __forceinline__ void wave_library(const LookupArgs &a, const int32_t *tidx,
                                             const float *tw, int lib, int64_t Lx, int m,
                                             const float *vs, const float *cs, const int *tgt,
                                             int Tn, int T) {
  const int S = tile_stride(T);
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (kSubs - 1);
  bool ok[TPL];
  int id[TPL];
  float c[TPL];
  float *pred[TPL];
#pragma unroll
  for (int u = 0; u < TPL; ++u) {
    const int t = sub * TPL + u;
    const bool in = sub * TPL < T && t < Tn;
    id[u] = in ? tgt[t] : 0;
    ok[u] = in && !(a.Ly_dev && a.Ly_dev[id[u]] < Lx);
    c[u] = in ? cs[t] : 0.0f;
    pred[u] = (TPL == 1 && ok[u] && a.pred) ? a.pred + static_cast<int64_t>(id[u]) * a.ldpred : nullptr;
  }
  Sums s[TPL];
  // predictions are written only with one target per lane (tiles of at most
  // 4 targets), which keeps the wider instantiations free of their registers
  if (TPL == 1 && a.pred)
    tile_pairs<K, TPL, TPL == 1>(tidx, tw, m, vs, T, S, pred, c, s);
  else
    tile_pairs<K, TPL, false>(tidx, tw, m, vs, T, S, pred, c, s);
  if (a.rho && lane < kSubs) {
#pragma unroll
    for (int u = 0; u < TPL; ++u)
      if (ok[u]) a.rho[static_cast<int64_t>(lib) * a.ldrho + id[u]] = pair_rho(m, s[u]);
  }
}

// Grid kernel: blockIdx.x = tile of T targets (bucket positions
// [x*T, x*T + T)), blockIdx.y = group of kWaves library slots from slot0;
// ms bounds every staged window (the dynamic LDS holds T * ms floats).
template <int K, int TPL>
__global__ __launch_bounds__(kThreads) void k_lookup(LookupArgs a, int T, int nslots, int slot0) {
  extern __shared__ float4 lds4[];
  float *vs = reinterpret_cast<float *>(lds4);
  __shared__ float cs[kLookupItemMaxTargets];
  __shared__ int tgt[kLookupItemMaxTargets];
  const int off = (a.E - 1) * a.tau + a.Tp;
  // targets of the launch: the host's list, or the bucket grouped on the device
  const bool dev = a.bucket_at != nullptr && a.tbl_off == nullptr;
  const int ntgt = dev ? a.bucket_at[a.E + 1] - a.bucket_at[a.E] : a.ntgt;
  const int32_t *tids = dev ? a.bucket_ids + a.bucket_at[a.E] : a.tgt_ids;
  // Host grid: blockIdx.x = tile, blockIdx.y = library group.  Device-bucket
  // grid (one dimension): workgroup i runs on XCD i % 8 (round-robin
  // dispatch); the kTileCols tile columns of a library group all go to one
  // XCD, so the workgroups an XCD runs together share two groups' tables in
  // its L2.
  int col = static_cast<int>(blockIdx.x), ncol = static_cast<int>(gridDim.x);
  int grp = static_cast<int>(blockIdx.y);
  if (dev) {
    const int i = static_cast<int>(blockIdx.x), k = i / kXcds;
    col = k % kTileCols;
    ncol = kTileCols;
    grp = kXcds * (k / kTileCols) + i % kXcds;
  }
  const int sbase = slot0 + grp * kWaves;
  const int lgT = 31 - __builtin_clz(T);
  int n_blk = 0;  // widest query range of the workgroup's libraries
  for (int w = 0; w < kWaves; ++w) {
    const int slot = sbase + w;
    if (slot >= slot0 + nslots) break;
    const int lib = a.lib_ids ? a.lib_ids[slot] : slot;
    const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
    const int mw = static_cast<int>(Lx) - off;
    n_blk = mw > n_blk ? mw : n_blk;
  }
  if (n_blk - 1 - 2 * a.excl < K) return;  // no table in this workgroup (uniform)

  const int wave = static_cast<int>(threadIdx.x) / kWave;
  const int slot = __builtin_amdgcn_readfirstlane(sbase + wave);
  const bool in = slot < slot0 + nslots;
  const int lib = in ? (a.lib_ids ? a.lib_ids[slot] : slot) : 0;
  const int64_t Lx = in ? (a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni) : 0;
  const int m = static_cast<int>(Lx) - off;
  const bool on = in && m - 1 - 2 * a.excl >= K;  // the table exists for this library
  const int64_t tbl = static_cast<int64_t>(slot) * a.tbl_stride;
  // tiles blockIdx.x, blockIdx.x + gridDim.x, ... (one per workgroup when the
  // host sized the grid to the target count)
  for (int tile = col; tile * T < ntgt; tile += ncol) {
    const int t0 = tile * T;
    const int Tn = ntgt - t0 < T ? ntgt - t0 : T;
    if (tile != col) __syncthreads();  // the previous tile is consumed
    if (static_cast<int>(threadIdx.x) < Tn)
      tgt[threadIdx.x] = tids ? tids[t0 + threadIdx.x] : t0 + static_cast<int>(threadIdx.x);
    stage_tile(a, tgt, Tn, T, lgT, off, n_blk, vs, cs);
    if (on) wave_library<K, TPL>(a, a.idx + tbl, a.w + tbl, lib, Lx, m, vs, cs, tgt, Tn, T);
  }
}

// Work-list kernel for one E (K = E + 1): persistent (counter != nullptr:
// workgroups pull items) or one workgroup per item.  An item stages a tile of
// targets once, over the window of its longest library, and wave w runs the
// item's library w against the tile.  Item fields are wave-uniform.
template <int K>
__global__ __launch_bounds__(kThreads) void k_lookup_items(LookupArgs a,
                                                            const LookupItem *__restrict__ items,
                                                            int n_items, int *counter) {
  extern __shared__ float4 lds4[];
  float *vs = reinterpret_cast<float *>(lds4);
  __shared__ float cs[kLookupItemMaxTargets];
  __shared__ int tgt[kLookupItemMaxTargets];
  __shared__ int item_s;
  const int E = K - 1;
  const int off = (E - 1) * a.tau + a.Tp;
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  for (int trip = 0;; ++trip) {
    int it;
    if (counter == nullptr) {
      if (trip > 0) break;
      it = static_cast<int>(blockIdx.x);
    } else {
      __syncthreads();  // the previous item is done with vs, cs, tgt and item_s
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
    const int lgT = 31 - __builtin_clz(T);
    // the first library of an item is its longest: its window covers all
    const int lib0 = __builtin_amdgcn_readfirstlane(a.item_libs[at]);
    const int ms = static_cast<int>((a.Lx_dev ? a.Lx_dev[lib0] : a.Lx_uni) - off);
    if (static_cast<int>(threadIdx.x) < Tn) tgt[threadIdx.x] = a.bucket_ids[a.bucket_at[E] + first + threadIdx.x];
    __syncthreads();
    if (ms < 1) continue;  // uniform: nothing of this item can be defined
    stage_tile(a, tgt, Tn, T, lgT, off, ms, vs, cs);
    if (wave < nlib) {  // uniform per wave
      const int lib = __builtin_amdgcn_readfirstlane(a.item_libs[at + wave]);
      const int64_t Lx = a.Lx_dev ? a.Lx_dev[lib] : a.Lx_uni;
      const int m = static_cast<int>(Lx) - off;
      if (m - 1 - 2 * a.excl >= K) {
        const int64_t o = a.tbl_off[static_cast<int64_t>(lib) * (EDM_E_MAX + 1) + E];
        if (T >= 16)
          wave_library<K, 4>(a, a.tbl_idx + o, a.tbl_w + o, lib, Lx, m, vs, cs, tgt, Tn, T);
        else if (T == 8)
          wave_library<K, 2>(a, a.tbl_idx + o, a.tbl_w + o, lib, Lx, m, vs, cs, tgt, Tn, T);
        else
          wave_library<K, 1>(a, a.tbl_idx + o, a.tbl_w + o, lib, Lx, m, vs, cs, tgt, Tn, T);
      }
    }
  }
}

// Centring constant of every target: float32 of the float64 mean over
// [0, Ly) (Ly_dev, or L_uni for all), one wave per target summing in a fixed
// order (lane-strided, then a butterfly), so every kernel and call that
// stages the target subtracts the same value.
__global__ __launch_bounds__(256) void k_target_means(const float *__restrict__ Y, int64_t ldy,
                                                      const int64_t *__restrict__ Ly_dev, int64_t L_uni,
                                                      int64_t N, float *__restrict__ cmean) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * (256 / kWave) + threadIdx.x / kWave;
  if (t >= N) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t L = Ly_dev ? Ly_dev[t] : L_uni;
  const float *__restrict__ y = Y + t * ldy;
  double sum = 0.0;
  for (int64_t i = lane; i < L; i += kWave) sum += static_cast<double>(y[i]);
#pragma unroll
  for (int msk = kWave / 2; msk > 0; msk >>= 1) sum += __shfl_xor(sum, msk);
  if (lane == 0) cmean[t] = L > 0 ? static_cast<float>(sum / static_cast<double>(L)) : 0.0f;
}

using LaunchFn = hipError_t (*)(const LookupArgs &, dim3, size_t, int, int, int, hipStream_t);

template <int K, int TPL>
hipError_t launch_k(const LookupArgs &a, dim3 grid, size_t shm, int T, int nslots, int slot0,
                    hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_lookup<K, TPL>);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_lookup<K, TPL>), grid, dim3(kThreads), shm, st, a, T, nslots, slot0);
  return hipGetLastError();
}

template <int TPL, size_t... I>
constexpr auto make_table(std::index_sequence<I...>) {
  return std::array<LaunchFn, sizeof...(I)>{&launch_k<static_cast<int>(I) + 1, TPL>...};
}

}  // namespace

hipError_t launch_target_means(const float *Y, int64_t ldy, const int64_t *Ly_dev, int64_t L_uni,
                               int64_t N, float *cmean, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  TimedLaunch timed(EDM_KF_LOOKUP, st);
  const int64_t blocks = (N + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_target_means, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, Y, ldy, Ly_dev,
                     L_uni, N, cmean);
  return hipGetLastError();
}

int lookup_tile_targets(int64_t m) {
  int T = kLookupItemMaxTargets;
  while (T > 1 && static_cast<int64_t>(tile_stride(T)) * m > kLdsFloats) T >>= 1;
  return T;
}

int64_t lookup_tile_floats(int T, int64_t m) { return static_cast<int64_t>(tile_stride(T)) * m; }

hipError_t launch_lookup(const LookupArgs &a, int nslots, int64_t m_max, hipStream_t st) {
  static const auto t4 = make_table<4>(std::make_index_sequence<EDM_K_MAX>{});
  static const auto t2 = make_table<2>(std::make_index_sequence<EDM_K_MAX>{});
  static const auto t1 = make_table<1>(std::make_index_sequence<EDM_K_MAX>{});
  if (nslots <= 0 || a.ntgt <= 0 || m_max <= 0) return hipSuccess;
  if (a.k < 1 || a.k > EDM_K_MAX || m_max > kLdsFloats) return hipErrorInvalidValue;
  int T = lookup_tile_targets(m_max);
  if (a.pred && T > 4) T = 4;                 // the prediction-writing form
  while (T > 1 && T / 2 >= a.ntgt) T >>= 1;  // no wider than the target count needs
  const size_t shm = static_cast<size_t>(lookup_tile_floats(T, m_max)) * sizeof(float);
  const unsigned gx = static_cast<unsigned>((a.ntgt + T - 1) / T);
  const auto &table = T >= 16 ? t4 : (T == 8 ? t2 : t1);
  TimedLaunch timed(EDM_KF_LOOKUP, st);
  constexpr int kMaxY = 32768 * kWaves;
  for (int s0 = 0; s0 < nslots; s0 += kMaxY) {
    const int ns = nslots - s0 < kMaxY ? nslots - s0 : kMaxY;
    const unsigned gy = static_cast<unsigned>((ns + kWaves - 1) / kWaves);
    hipError_t e = table[a.k - 1](a, dim3(gx, gy), shm, T, ns, s0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_lookup_bucket(const LookupArgs &a, int nslots, int64_t m_max, int64_t n_tgt_max,
                                hipStream_t st) {
  static const auto t4 = make_table<4>(std::make_index_sequence<EDM_K_MAX>{});
  static const auto t2 = make_table<2>(std::make_index_sequence<EDM_K_MAX>{});
  static const auto t1 = make_table<1>(std::make_index_sequence<EDM_K_MAX>{});
  if (nslots <= 0 || n_tgt_max <= 0 || m_max <= 0) return hipSuccess;
  if (a.k < 1 || a.k > EDM_K_MAX || m_max > kLdsFloats || !a.bucket_at || !a.bucket_ids || a.tbl_off ||
      a.pred)
    return hipErrorInvalidValue;
  int T = lookup_tile_targets(m_max);
  while (T > 1 && T / 2 >= n_tgt_max) T >>= 1;
  const size_t shm = static_cast<size_t>(lookup_tile_floats(T, m_max)) * sizeof(float);
  // kTileCols tile columns per library group, each workgroup walking its
  // column's tiles; library groups padded to a multiple of the XCD count
  // (the kernel maps workgroups to groups XCD by XCD)
  const auto &table = T >= 16 ? t4 : (T == 8 ? t2 : t1);
  TimedLaunch timed(EDM_KF_LOOKUP, st);
  constexpr int kMaxSlots = 65536 * kWaves;
  for (int s0 = 0; s0 < nslots; s0 += kMaxSlots) {
    const int ns = nslots - s0 < kMaxSlots ? nslots - s0 : kMaxSlots;
    const int64_t groups = (ns + kWaves - 1) / kWaves;
    const int64_t padded = (groups + kXcds - 1) / kXcds * kXcds;
    hipError_t e = table[a.k - 1](a, dim3(static_cast<unsigned>(padded * kTileCols), 1), shm, T, ns, s0, st);
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
  if (E < 1 || E > EDM_E_MAX || lds_floats > kLdsFloats) return hipErrorInvalidValue;
  const size_t shm = static_cast<size_t>(lds_floats) * sizeof(float);
  const void *fn = reinterpret_cast<const void *>(fns[E - 1]);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  TimedLaunch timed(EDM_KF_LOOKUP, st);
  if (wg_per_cu <= 0) {
    hipLaunchKernelGGL(fns[E - 1], dim3(static_cast<unsigned>(n_items)), dim3(kThreads), shm,
                       st, a, items, n_items, static_cast<int *>(nullptr));
  } else {
    int grid = wg_per_cu * n_cu;
    if (grid > n_items) grid = n_items;
    hipLaunchKernelGGL(fns[E - 1], dim3(static_cast<unsigned>(grid)), dim3(kThreads), shm, st,
                       a, items, n_items, counter);
  }
  return hipGetLastError();
}

}  // namespace edm
