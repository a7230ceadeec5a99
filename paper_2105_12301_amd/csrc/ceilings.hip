// Empirical ceilings of the chip, measured with this library's own kernels
// (the paper builds its rooflines from measured ceilings, Section 4.4): HBM
// streaming bandwidth (a vectorised copy of a buffer far larger than the
// caches), BF16 matrix-core throughput (independent chains of
// v_mfma_f32_32x32x16_bf16 on register operands) and float32 vector throughput
// (independent non-fused additions, the operation mix of the neighbour key).
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/edm.h"
#include "ctx.h"

#pragma clang fp contract(off)

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                              int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

constexpr int kMfmaChains = 4;

__global__ __launch_bounds__(256) void k_mfma(int iters, float seed, float *__restrict__ out) {
  bf16x8_t a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = static_cast<__bf16>(seed * (threadIdx.x + i));
    b[i] = static_cast<__bf16>(seed * (threadIdx.x - i));
  }
  f32x16_t c[kMfmaChains];
#pragma unroll
  for (int k = 0; k < kMfmaChains; ++k) c[k] = f32x16_t{};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kMfmaChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[k], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kMfmaChains; ++k)
#pragma unroll
    for (int v = 0; v < 16; ++v) s += c[k][v];
  if (s == 1234.5f) out[threadIdx.x] = s;  // keeps the chains alive
}

constexpr int kValuChains = 8;

__global__ __launch_bounds__(256) void k_valu(int iters, float seed, float *__restrict__ out) {
  float acc[kValuChains];
#pragma unroll
  for (int k = 0; k < kValuChains; ++k) acc[k] = seed * (threadIdx.x + k);
  const float d = seed * 1e-7f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kValuChains; ++k) acc[k] = acc[k] + d;
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kValuChains; ++k) s += acc[k];
  if (s == 1234.5f) out[threadIdx.x] = s;
}

}  // namespace

using namespace edm::host;

extern "C" int edm_ceilings(edm_ctx *ctx, double *hbm_gbps, double *mfma_bf16_tflops,
                            double *valu_fp32_tops) {
  EDM_RC(check_ctx(ctx));
  if (!hbm_gbps || !mfma_bf16_tflops || !valu_fp32_tops) return set_err(ctx, EDM_E_ARG, "NULL output");
  int dev = 0, n_cu = 0;
  EDM_HIP(ctx, hipGetDevice(&dev));
  EDM_HIP(ctx, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  // 2 x 2 GiB: far beyond the caches (and the 256 MB last-level cache)
  const size_t half = size_t(2) << 30;
  EDM_RC(ws_reserve(ctx, 2 * half));
  const int64_t n4 = static_cast<int64_t>(half / sizeof(float4));
  const float4 *src = reinterpret_cast<const float4 *>(ctx->ws);
  float4 *dst = reinterpret_cast<float4 *>(ctx->ws + half);
  float *sink = reinterpret_cast<float *>(ctx->ws);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EDM_HIP(ctx, hipEventCreate(&e0));
  EDM_HIP(ctx, hipEventCreate(&e1));
  auto timed = [&](auto launch, int reps, float &ms) -> int {
    launch();  // warm-up
    EDM_HIP(ctx, hipGetLastError());
    EDM_HIP(ctx, hipEventRecord(e0, ctx->stream));
    for (int r = 0; r < reps; ++r) launch();
    EDM_HIP(ctx, hipEventRecord(e1, ctx->stream));
    EDM_HIP(ctx, hipEventSynchronize(e1));
    EDM_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    return EDM_OK;
  };
  float ms = 0.0f;
  int rc = timed([&] { hipLaunchKernelGGL(k_copy, dim3(n_cu * 64), dim3(256), 0, ctx->stream, src, dst, n4); },
                 10, ms);
  if (rc == EDM_OK) {
    *hbm_gbps = 2.0 * static_cast<double>(half) / (ms * 1e-3) / 1e9;
    const int iters = 4096;
    const int blocks = n_cu * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    rc = timed([&] { hipLaunchKernelGGL(k_mfma, dim3(blocks), dim3(256), 0, ctx->stream, iters, 1e-3f, sink); },
               5, ms);
    if (rc == EDM_OK) {
      const double flops = 2.0 * 32 * 32 * 16 * kMfmaChains * static_cast<double>(iters) * blocks * 4;
      *mfma_bf16_tflops = flops / (ms * 1e-3) / 1e12;
      const int vit = 1 << 16;
      rc = timed([&] { hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(256), 0, ctx->stream, vit, 1e-3f, sink); },
                 5, ms);
      if (rc == EDM_OK) {
        const double ops = static_cast<double>(kValuChains) * vit * blocks * 256;
        *valu_fp32_tops = ops / (ms * 1e-3) / 1e12;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
