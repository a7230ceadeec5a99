// Learned embedding-dimension surrogate: kernels for training (float32) and
// inference of a small 1-D convolutional network.
//
// The network (labels come from the simplex E sweep, the method's own E
// selection of Section 2.1 step 1 / Section 3.4 of the kEDM paper):
//   x[L] -> conv(1->C, KW) -> ReLU -> conv(C->C, KW) -> ReLU -> conv(C->C, KW)
//        -> ReLU -> mean over time -> linear(C->20) -> logits over E = 1..20
// with zero "same" padding.  Activations are [B][C][L] row-major.
//
// Convolutions are tiled for one workgroup = one series x 128 time steps x all
// output channels: the input window (channel chunk x (128 + KW - 1)) and the
// weight chunk are staged in LDS, and each thread accumulates a 4-channel x
// 8-step register tile (224 FMAs per 42 LDS reads).  The backward pass over
// the data is the same contraction with the weights transposed and flipped in
// the staging step and the ReLU mask of the previous layer applied on output.
// Weight gradients reduce over (series, time) in slices with a second pass
// over the slices, so no float atomics are involved and results are
// deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/edm.h"
#include "net_kernels.h"

namespace edm {
namespace {

constexpr int KW = EDM_NET_KW;
constexpr int HALO = KW / 2;
constexpr int TT = 128;   // time steps per workgroup
constexpr int CCH = 16;   // input channels staged per chunk
constexpr int NCLS = EDM_NET_CLASSES;

// MODE 0: y = relu(conv(x, w) + b)                  (forward)
// MODE 1: y = conv(x, w^T flipped) * (aprev > 0)    (backward over the data)
// MODE 2: y = conv(x, w) + b                        (forward without ReLU; tests)
template <int MODE>
__global__ __launch_bounds__(256) void k_conv(const float *__restrict__ x, int64_t ldx_b,
                                              int64_t ldx_c, int Ci, int Co, int L,
                                              const float *__restrict__ w,
                                              const float *__restrict__ bias,
                                              const float *__restrict__ aprev,
                                              float *__restrict__ y) {
  __shared__ float xs[CCH][TT + KW - 1];
  __shared__ float ws[64][CCH][KW];
  const int b = blockIdx.y;
  const int t0 = blockIdx.x * TT;
  const int tid = threadIdx.x;
  const int ty = tid >> 4;  // 16 groups of 4 output channels
  const int tx = tid & 15;  // 16 groups of 8 time steps
  float acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0f;

  const float *xb = x + static_cast<int64_t>(b) * ldx_b;
  for (int c0 = 0; c0 < Ci; c0 += CCH) {
    const int cn = Ci - c0 < CCH ? Ci - c0 : CCH;
    __syncthreads();
    for (int e = tid; e < CCH * (TT + KW - 1); e += 256) {
      const int c = e / (TT + KW - 1), t = e - c * (TT + KW - 1);
      const int tg = t0 + t - HALO;
      float v = 0.0f;
      if (c < cn && tg >= 0 && tg < L) v = xb[static_cast<int64_t>(c0 + c) * ldx_c + tg];
      xs[c][t] = v;
    }
    for (int e = tid; e < 64 * CCH * KW; e += 256) {
      const int o = e / (CCH * KW), r = e - o * (CCH * KW);
      const int c = r / KW, k = r - c * KW;
      float v = 0.0f;
      if (o < Co && c < cn) {
        if (MODE == 1)  // w_eff[o][i][k] = w[i][o][KW-1-k], w is [Ci_fwd = Co][Co_fwd = Ci][KW]
          v = w[(static_cast<int64_t>(c0 + c) * Co + o) * KW + (KW - 1 - k)];
        else
          v = w[(static_cast<int64_t>(o) * Ci + (c0 + c)) * KW + k];
      }
      ws[o][c][k] = v;
    }
    __syncthreads();
    for (int c = 0; c < cn; ++c) {
      float xv[8 + KW - 1];
#pragma unroll
      for (int j = 0; j < 8 + KW - 1; ++j) xv[j] = xs[c][tx * 8 + j];
#pragma unroll
      for (int k = 0; k < KW; ++k) {
        float wv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) wv[i] = ws[ty * 4 + i][c][k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(wv[i], xv[j + k], acc[i][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = ty * 4 + i;
    if (o >= Co) continue;
    const float bo = (MODE != 1 && bias) ? bias[o] : 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int t = t0 + tx * 8 + j;
      if (t >= L) continue;
      const int64_t at = (static_cast<int64_t>(b) * Co + o) * L + t;
      float v = acc[i][j] + bo;
      if (MODE == 0) v = fmaxf(v, 0.0f);
      if (MODE == 1) v = aprev[at] > 0.0f ? v : 0.0f;
      y[at] = v;
    }
  }
}

// ---- BF16 inference form of the C -> C convolutions (matrix cores) --------
// The contraction over (tap k, input channel i) runs as a GEMM on
// v_mfma_f32_32x32x16_bf16: A = weights [co][k*C + i] (BF16), B = the input
// window [k*C + i][t] = x[i][t + k - HALO] (BF16), FP32 accumulation.  One
// workgroup = one series x 256 time steps x all C output channels; the input
// window is staged in LDS transposed to [t][i] so every lane's eight K values
// (eight consecutive channels at one tap) are one aligned 16-byte read, and
// the weights are staged as [co][k][i].  Wave w owns time tiles 2w, 2w+1 and
// every output-channel tile.  Rows are padded by 8 BF16 values (16 bytes)
// against LDS bank conflicts.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int TB = 256;  // time steps per workgroup of the BF16 convolution

__device__ __forceinline__ uint16_t to_bf16(float f) {  // round to nearest even (finite f)
  const uint32_t u = __float_as_uint(f);
  return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// w[co][ci][k] float32 -> wb[co][k][ci] BF16.
__global__ void k_w_to_bf16(const float *__restrict__ w, int C, uint16_t *__restrict__ wb) {
  const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= C * C * KW) return;
  const int co = i / (KW * C), r = i - co * (KW * C);
  const int k = r / C, ci = r - k * C;
  wb[i] = to_bf16(w[(co * C + ci) * KW + k]);
}

template <int C>
constexpr size_t conv_bf16_lds() {
  return sizeof(uint16_t) * ((TB + KW - 1) * (C + 8) + C * (KW * C + 8));
}

// y = relu(conv(x, w) + b) for x, y [B][C][L] float32 (inputs rounded to BF16).
template <int C>
__global__ __launch_bounds__(256) void k_conv_bf16(const float *__restrict__ x, int L,
                                                   const uint16_t *__restrict__ wb,
                                                   const float *__restrict__ bias,
                                                   float *__restrict__ y) {
  static_assert(C % 32 == 0 && C <= 64, "C must be 32 or 64");
  constexpr int XR = TB + KW - 1, XS = C + 8, WR = KW * C, WS = WR + 8;
  constexpr int NCO = C / 32, NCC = C / 16;
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_bf16[];
  uint16_t *xs = lds_bf16;
  uint16_t *ws = lds_bf16 + XR * XS;
  const int b = blockIdx.y;
  const int t0 = blockIdx.x * TB;
  const int tid = threadIdx.x;
  const float *xb = x + static_cast<int64_t>(b) * C * L;
  for (int e = tid; e < C * WR; e += 256) {
    const int co = e / WR, r = e - co * WR;
    ws[co * WS + r] = wb[e];
  }
  for (int e = tid; e < C * XR; e += 256) {
    const int ci = e / XR, t = e - ci * XR;
    const int tg = t0 + t - HALO;
    const float v = (tg >= 0 && tg < L) ? xb[static_cast<int64_t>(ci) * L + tg] : 0.0f;
    xs[t * XS + ci] = to_bf16(v);
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, n = lane & 31, h = lane >> 5;
  f32x16_t acc[2][NCO];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int c = 0; c < NCO; ++c) acc[j][c] = f32x16_t{};
#pragma unroll 1
  for (int k = 0; k < KW; ++k) {
#pragma unroll
    for (int cc = 0; cc < NCC; ++cc) {
      bf16x8_t bop[2], aop[NCO];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int tl = 64 * wave + 32 * j + n;
        bop[j] = *reinterpret_cast<const bf16x8_t *>(xs + (tl + k) * XS + 16 * cc + 8 * h);
      }
#pragma unroll
      for (int c = 0; c < NCO; ++c)
        aop[c] = *reinterpret_cast<const bf16x8_t *>(ws + (32 * c + n) * WS + k * C + 16 * cc + 8 * h);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int c = 0; c < NCO; ++c)
          acc[j][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[c], bop[j], acc[j][c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int t = t0 + 64 * wave + 32 * j + n;
    if (t >= L) continue;
#pragma unroll
    for (int c = 0; c < NCO; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int co = 32 * c + 8 * (v >> 2) + 4 * h + (v & 3);
        y[(static_cast<int64_t>(b) * C + co) * L + t] = fmaxf(acc[j][c][v] + bias[co], 0.0f);
      }
  }
}

// Partial weight gradients of one slice of (series, time):
// part[s][o][i][k] = sum over the slice of dz[b][o][t] * x[b][i][t + k - HALO],
// part_b[s][o] = sum over the slice of dz[b][o][t] (from the i-chunk-0 blocks).
// Block = 8 input channels x all (<= 64) output channels; 256 threads =
// 16 output groups (4 channels) x 4 input pairs x 4 time quarters.
constexpr int WT = 64;  // time steps staged per tile
__global__ __launch_bounds__(256) void k_conv_wgrad(const float *__restrict__ x, int64_t ldx_b,
                                                    int64_t ldx_c, int Ci, int Co, int L, int B,
                                                    const float *__restrict__ dz,
                                                    int64_t tiles_per_slice,
                                                    float *__restrict__ part,
                                                    float *__restrict__ part_b) {
  __shared__ float ds[64][WT];
  __shared__ float xs2[8][WT + KW - 1];
  __shared__ float red[64 * 4 * 2 * KW];  // one quarter's accumulators
  const int ic0 = blockIdx.x * 8;
  const int slice = blockIdx.y;
  const int tid = threadIdx.x;
  const int og = tid & 15, ip = (tid >> 4) & 3, tq = tid >> 6;
  float acc[4][2][KW];
  float accb[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    accb[a] = 0.0f;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < KW; ++k) acc[a][c][k] = 0.0f;
  }
  const int tiles_per_series = (L + WT - 1) / WT;
  const int64_t total_tiles = static_cast<int64_t>(B) * tiles_per_series;
  const int64_t tile_begin = static_cast<int64_t>(slice) * tiles_per_slice;
  int64_t tile_end = tile_begin + tiles_per_slice;
  if (tile_end > total_tiles) tile_end = total_tiles;
  for (int64_t tile = tile_begin; tile < tile_end; ++tile) {
    const int b = static_cast<int>(tile / tiles_per_series);
    const int t0 = static_cast<int>(tile - static_cast<int64_t>(b) * tiles_per_series) * WT;
    __syncthreads();
    for (int e = tid; e < 64 * WT; e += 256) {
      const int o = e / WT, t = e - o * WT;
      float v = 0.0f;
      if (o < Co && t0 + t < L) v = dz[(static_cast<int64_t>(b) * Co + o) * L + t0 + t];
      ds[o][t] = v;
    }
    for (int e = tid; e < 8 * (WT + KW - 1); e += 256) {
      const int c = e / (WT + KW - 1), t = e - c * (WT + KW - 1);
      const int tg = t0 + t - HALO;
      float v = 0.0f;
      if (ic0 + c < Ci && tg >= 0 && tg < L)
        v = x[static_cast<int64_t>(b) * ldx_b + static_cast<int64_t>(ic0 + c) * ldx_c + tg];
      xs2[c][t] = v;
    }
    __syncthreads();
    const int tb = tq * (WT / 4);
    float win[2][KW];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < KW - 1; ++k) win[c][k] = xs2[ip * 2 + c][tb + k];
    for (int tt = 0; tt < WT / 4; ++tt) {
      const int t = tb + tt;
#pragma unroll
      for (int c = 0; c < 2; ++c) win[c][KW - 1] = xs2[ip * 2 + c][t + KW - 1];
      float dv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) dv[a] = ds[og * 4 + a][t];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        accb[a] += dv[a];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int k = 0; k < KW; ++k) acc[a][c][k] = fmaf(dv[a], win[c][k], acc[a][c][k]);
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < KW - 1; ++k) win[c][k] = win[c][k + 1];
    }
  }
  // reduce the 4 time quarters through LDS (one quarter per round), then
  // write this slice's partials
  constexpr int per = 4 * 2 * KW;  // accumulators per thread
  const int lt = tid & 63;         // thread index within its quarter
  for (int q = 1; q < 4; ++q) {
    __syncthreads();
    if (tq == q) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int k = 0; k < KW; ++k) red[lt * per + (a * 2 + c) * KW + k] = acc[a][c][k];
    }
    __syncthreads();
    if (tq == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int k = 0; k < KW; ++k) acc[a][c][k] += red[lt * per + (a * 2 + c) * KW + k];
    }
  }
  if (tq == 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < KW; ++k) {
          const int o = og * 4 + a, i = ic0 + ip * 2 + c;
          if (o < Co && i < Ci)
            part[((static_cast<int64_t>(slice) * Co + o) * Ci + i) * KW + k] = acc[a][c][k];
        }
  }
  // bias partials (first input chunk only): sum over the time quarters of
  // the ip == 0 threads, which hold output channel o at og = o / 4, a = o % 4
  __syncthreads();
  if (blockIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a) red[tid * 4 + a] = ip == 0 ? accb[a] : 0.0f;
    __syncthreads();
    if (tid < 64) {
      const int o = tid;
      float v = 0.0f;
      for (int q = 0; q < 4; ++q) v += red[(q * 64 + (o >> 2)) * 4 + (o & 3)];
      if (o < Co) part_b[static_cast<int64_t>(slice) * Co + o] = v;
    }
  }
}

__global__ void k_sum_slices(const float *__restrict__ part, int64_t n, int slices,
                             float *__restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = 0.0f;
  for (int s = 0; s < slices; ++s) v += part[static_cast<int64_t>(s) * n + i];
  out[i] = v;
}

// g[b][c] = mean_t a[b][c][t]; logits[b][j] = bo[j] + sum_c wo[j][c] g[b][c].
// One workgroup per series.
__global__ __launch_bounds__(256) void k_pool_linear(const float *__restrict__ a, int C, int L,
                                                     const float *__restrict__ wo,
                                                     const float *__restrict__ bo,
                                                     float *__restrict__ g,
                                                     float *__restrict__ logits) {
  __shared__ float gs[64];
  const int b = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = wave; c < C; c += 4) {
    const float *row = a + (static_cast<int64_t>(b) * C + c) * L;
    float s = 0.0f;
    for (int t = lane; t < L; t += 64) s += row[t];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) {
      gs[c] = s / static_cast<float>(L);
      g[static_cast<int64_t>(b) * C + c] = s / static_cast<float>(L);
    }
  }
  __syncthreads();
  if (threadIdx.x < NCLS) {
    const int j = threadIdx.x;
    float v = bo[j];
    for (int c = 0; c < C; ++c) v = fmaf(wo[j * C + c], gs[c], v);
    logits[static_cast<int64_t>(b) * NCLS + j] = v;
  }
}

// Softmax cross-entropy per series: loss_b[b], dlog[b][j] = (p_j - [j == y]) / B.
__global__ void k_softmax_ce(const float *__restrict__ logits, const int32_t *__restrict__ labels,
                             int B, float *__restrict__ loss_b, float *__restrict__ dlog) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float *z = logits + static_cast<int64_t>(b) * NCLS;
  float mx = z[0];
  for (int j = 1; j < NCLS; ++j) mx = fmaxf(mx, z[j]);
  float s = 0.0f;
  for (int j = 0; j < NCLS; ++j) s += expf(z[j] - mx);
  int y = labels[b] - 1;
  y = y < 0 ? 0 : (y >= NCLS ? NCLS - 1 : y);  // labels are validated on the host
  loss_b[b] = logf(s) - (z[y] - mx);
  for (int j = 0; j < NCLS; ++j)
    dlog[static_cast<int64_t>(b) * NCLS + j] = (expf(z[j] - mx) / s - (j == y ? 1.0f : 0.0f)) / B;
}

// Linear + pool backward.  Output-layer gradients (one thread per weight),
// then dz3[b][c][t] = dg[b][c] / L * (a3 > 0) over the activations.
__global__ void k_linear_bwd(const float *__restrict__ dlog, const float *__restrict__ g, int B,
                             int C, float *__restrict__ dwo, float *__restrict__ dbo) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < NCLS * C) {
    const int j = e / C, c = e - j * C;
    float v = 0.0f;
    for (int b = 0; b < B; ++b) v = fmaf(dlog[b * NCLS + j], g[static_cast<int64_t>(b) * C + c], v);
    dwo[e] = v;
  } else if (e < NCLS * C + NCLS) {
    const int j = e - NCLS * C;
    float v = 0.0f;
    for (int b = 0; b < B; ++b) v += dlog[b * NCLS + j];
    dbo[j] = v;
  }
}

__global__ void k_pool_bwd(const float *__restrict__ dlog, const float *__restrict__ wo,
                           const float *__restrict__ a3, int64_t B, int C, int L,
                           float *__restrict__ dz3) {
  const int64_t total = B * C * L;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t bc = e / L;
    const int b = static_cast<int>(bc / C), c = static_cast<int>(bc - static_cast<int64_t>(b) * C);
    float dg = 0.0f;
#pragma unroll
    for (int j = 0; j < NCLS; ++j) dg = fmaf(dlog[b * NCLS + j], wo[j * C + c], dg);
    dz3[e] = a3[e] > 0.0f ? dg / static_cast<float>(L) : 0.0f;
  }
}

__global__ void k_mean(const float *__restrict__ v, int n, float *__restrict__ out) {
  __shared__ float s[256];
  float a = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) a += v[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int m = 128; m > 0; m >>= 1) {
    if (static_cast<int>(threadIdx.x) < m) s[threadIdx.x] += s[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0] / static_cast<float>(n);
}

// Adam (Kingma & Ba) with bias correction.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks_for(int64_t n, int t) {
  int64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<unsigned>(b);
}

}  // namespace

int64_t net_param_count(int C) { return static_cast<int64_t>(KW) * C + C + 2 * (static_cast<int64_t>(C) * C * KW + C) + NCLS * C + NCLS; }

NetParams net_params(const float *theta, int C) {
  NetParams p;
  const float *q = theta;
  p.w1 = q; q += static_cast<int64_t>(C) * KW;
  p.b1 = q; q += C;
  p.w2 = q; q += static_cast<int64_t>(C) * C * KW;
  p.b2 = q; q += C;
  p.w3 = q; q += static_cast<int64_t>(C) * C * KW;
  p.b3 = q; q += C;
  p.wo = q; q += static_cast<int64_t>(NCLS) * C;
  p.bo = q;
  return p;
}

int64_t net_workspace_floats(int C, int64_t B, int64_t L) {
  // a1, a2, a3, dz (x2), g, logits, dlog, loss_b, partials
  return 5 * B * C * L + B * C + 3 * B * NCLS + B + kNetSlices * (static_cast<int64_t>(C) * C * KW + C) + 64;
}

hipError_t net_forward(const float *theta, int C, const float *X, int64_t B, int64_t L,
                       int64_t ldx, float *ws, float *logits, hipStream_t st) {
  const NetParams P = net_params(theta, C);
  float *a1 = ws, *a2 = a1 + B * C * L, *a3 = a2 + B * C * L;
  float *g = a3 + 3 * B * C * L;  // after a3 and the two dz buffers
  const dim3 grid(static_cast<unsigned>((L + TT - 1) / TT), static_cast<unsigned>(B));
  hipLaunchKernelGGL(k_conv<0>, grid, dim3(256), 0, st, X, ldx, 0, 1, C, static_cast<int>(L), P.w1, P.b1, nullptr, a1);
  hipLaunchKernelGGL(k_conv<0>, grid, dim3(256), 0, st, a1, C * L, L, C, C, static_cast<int>(L), P.w2, P.b2, nullptr, a2);
  hipLaunchKernelGGL(k_conv<0>, grid, dim3(256), 0, st, a2, C * L, L, C, C, static_cast<int>(L), P.w3, P.b3, nullptr, a3);
  hipLaunchKernelGGL(k_pool_linear, dim3(static_cast<unsigned>(B)), dim3(256), 0, st, a3, C, static_cast<int>(L), P.wo, P.bo, g, logits);
  return hipGetLastError();
}

template <int C>
hipError_t conv_bf16_layer(const float *in, int64_t B, int64_t L, const uint16_t *wb,
                           const float *bias, float *out, hipStream_t st) {
  const void *fn = reinterpret_cast<const void *>(&k_conv_bf16<C>);
  const size_t shm = conv_bf16_lds<C>();
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm));
  if (e != hipSuccess) return e;
  const dim3 grid(static_cast<unsigned>((L + TB - 1) / TB), static_cast<unsigned>(B));
  hipLaunchKernelGGL(k_conv_bf16<C>, grid, dim3(256), shm, st, in, static_cast<int>(L), wb, bias, out);
  return hipGetLastError();
}

hipError_t net_forward_bf16(const float *theta, int C, const float *X, int64_t B, int64_t L,
                            int64_t ldx, float *ws, float *logits, hipStream_t st) {
  if (C != 32 && C != 64) return hipErrorInvalidValue;
  const NetParams P = net_params(theta, C);
  float *a1 = ws, *a2 = a1 + B * C * L, *a3 = a2 + B * C * L;
  float *g = a3 + B * C * L;
  uint16_t *wb2 = reinterpret_cast<uint16_t *>(g + B * C);
  uint16_t *wb3 = wb2 + C * C * KW;
  const unsigned nw = static_cast<unsigned>((C * C * KW + 255) / 256);
  hipLaunchKernelGGL(k_w_to_bf16, dim3(nw), dim3(256), 0, st, P.w2, C, wb2);
  hipLaunchKernelGGL(k_w_to_bf16, dim3(nw), dim3(256), 0, st, P.w3, C, wb3);
  const dim3 grid(static_cast<unsigned>((L + TT - 1) / TT), static_cast<unsigned>(B));
  hipLaunchKernelGGL(k_conv<0>, grid, dim3(256), 0, st, X, ldx, 0, 1, C, static_cast<int>(L), P.w1, P.b1, nullptr, a1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = C == 64 ? conv_bf16_layer<64>(a1, B, L, wb2, P.b2, a2, st) : conv_bf16_layer<32>(a1, B, L, wb2, P.b2, a2, st);
  if (e != hipSuccess) return e;
  e = C == 64 ? conv_bf16_layer<64>(a2, B, L, wb3, P.b3, a3, st) : conv_bf16_layer<32>(a2, B, L, wb3, P.b3, a3, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pool_linear, dim3(static_cast<unsigned>(B)), dim3(256), 0, st, a3, C, static_cast<int>(L), P.wo, P.bo, g, logits);
  return hipGetLastError();
}

hipError_t net_loss_grad(const float *theta, int C, const float *X, const int32_t *labels,
                         int64_t B, int64_t L, int64_t ldx, float *ws, float *loss,
                         float *grad, hipStream_t st) {
  const NetParams P = net_params(theta, C);
  float *a1 = ws, *a2 = a1 + B * C * L, *a3 = a2 + B * C * L;
  float *dzA = a3 + B * C * L, *dzB = dzA + B * C * L;
  float *g = dzB + B * C * L, *logits = g + B * C, *dlog = logits + B * NCLS;
  float *loss_b = dlog + B * NCLS;
  float *part = loss_b + B;
  float *part_b = part + static_cast<int64_t>(kNetSlices) * C * C * KW;
  hipError_t e = net_forward(theta, C, X, B, L, ldx, ws, logits, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_softmax_ce, dim3(blocks_for(B, 128)), dim3(128), 0, st, logits, labels, static_cast<int>(B), loss_b, dlog);
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, loss_b, static_cast<int>(B), loss);
  const NetParams G = net_params(grad, C);
  float *dwo = const_cast<float *>(G.wo), *dbo = const_cast<float *>(G.bo);
  hipLaunchKernelGGL(k_linear_bwd, dim3(blocks_for(NCLS * C + NCLS, 256)), dim3(256), 0, st, dlog, g, static_cast<int>(B), C, dwo, dbo);
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for(B * C * L, 256)), dim3(256), 0, st, dlog, P.wo, a3, B, C, static_cast<int>(L), dzA);

  const int tiles = static_cast<int>(B * ((L + WT - 1) / WT));
  const int64_t tps = (tiles + kNetSlices - 1) / kNetSlices;
  const dim3 cgrid(static_cast<unsigned>((L + TT - 1) / TT), static_cast<unsigned>(B));
  struct Layer { const float *in; int64_t ldb, ldc; int Ci; const float *w; float *dw; float *db; };
  const Layer layers[3] = {
      {a2, C * L, L, C, P.w3, const_cast<float *>(G.w3), const_cast<float *>(G.b3)},
      {a1, C * L, L, C, P.w2, const_cast<float *>(G.w2), const_cast<float *>(G.b2)},
      {X, ldx, 0, 1, P.w1, const_cast<float *>(G.w1), const_cast<float *>(G.b1)}};
  float *dz = dzA, *dz_next = dzB;
  for (int l = 0; l < 3; ++l) {
    const Layer &Ly = layers[l];
    hipLaunchKernelGGL(k_conv_wgrad, dim3(static_cast<unsigned>((Ly.Ci + 7) / 8), kNetSlices), dim3(256), 0, st,
                       Ly.in, Ly.ldb, Ly.ldc, Ly.Ci, C, static_cast<int>(L), static_cast<int>(B), dz, tps, part, part_b);
    const int64_t nw = static_cast<int64_t>(C) * Ly.Ci * KW;
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(nw, 256)), dim3(256), 0, st, part, nw, kNetSlices, Ly.dw);
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(C, 256)), dim3(256), 0, st, part_b, static_cast<int64_t>(C), kNetSlices, Ly.db);
    if (l < 2) {  // gradient with respect to this layer's input, masked by its ReLU
      hipLaunchKernelGGL(k_conv<1>, cgrid, dim3(256), 0, st, dz, C * L, L, C, C, static_cast<int>(L), Ly.w, nullptr, Ly.in, dz_next);
      float *t = dz; dz = dz_next; dz_next = t;
    }
  }
  return hipGetLastError();
}

hipError_t net_adam(float *p, const float *g, float *m, float *v, int64_t n, int step, float lr,
                    float b1, float b2, float eps, hipStream_t st) {
  const float c1 = 1.0f - powf(b1, static_cast<float>(step));
  const float c2 = 1.0f - powf(b2, static_cast<float>(step));
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace edm
