// Allocation-free form of edm_simplex_sweep for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid hipMalloc): its scratch (series lengths and the per-block Pearson
// co-moments of the self-predictions) lives in one file-scope device array
// of kNoAllocScratchBytes per GPU instead of the context's growable
// workspace.  Every call on a GPU shares that GPU's array, so calls that
// overlap in time on one GPU race; the array keeps the last call's contents
// (nothing in it needs to start at zero: every co-moment the epilogue reads
// is written by the scan of the same call).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/edm.h"
#include "ctx.h"
#include "kernels.h"
#include "validate.h"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

__global__ void k_fill_lengths(int64_t *__restrict__ out, int64_t n, int64_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = v;
}

std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace edm {
namespace host {

// Device address of this GPU's copy of the scratch array (the host-side name
// of the array is not a device address).  Resolved once per device, with that
// device current; called from edm_ctx_create.
int noalloc_scratch_init(edm_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_err(ctx, EDM_E_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[ctx->device]) return EDM_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    return hip_err(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  }
  g_scratch_ptr[ctx->device] = static_cast<char *>(p);
  return EDM_OK;
}

}  // namespace host
}  // namespace edm

using namespace edm::host;

extern "C" int edm_simplex_sweep_noalloc(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N,
                                         int64_t ldx, int32_t E_max, int32_t tau, int32_t Tp,
                                         float *rho, int32_t *E_opt) {
  std::string msg;
  const int rc = edm::check_sweep(X, L, N, ldx, E_max, tau, Tp, rho, E_opt, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (N == 0) return EDM_OK;
  if (N > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");
  char *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
  }
  if (!base) return set_err(ctx, EDM_E_HIP, "static scratch not resolved for this device");
  const int64_t L_max = *std::max_element(L, L + N);
  const int32_t mom_blocks = static_cast<int32_t>((L_max + edm::kKnnThreads - 1) / edm::kKnnThreads);
  Plan plan;
  const size_t off_L = plan.take(sizeof(int64_t) * static_cast<size_t>(N));
  const size_t off_mom = plan.take(edm::kMomBytes * static_cast<size_t>(N) * E_max * mom_blocks);
  if (plan.bytes > kNoAllocScratchBytes)
    return set_err(ctx, EDM_E_NOMEM,
                   "edm_simplex_sweep_noalloc needs " + std::to_string(plan.bytes) +
                       " bytes of scratch (N * E_max * ceil(L_max/256) * 48 + 8 N), above its static " +
                       std::to_string(kNoAllocScratchBytes) + " bytes: use edm_simplex_sweep");
  int64_t *L_dev = reinterpret_cast<int64_t *>(base + off_L);
  edm::Mom *mom = reinterpret_cast<edm::Mom *>(base + off_mom);
  if (std::all_of(L, L + N, [&](int64_t v) { return v == L[0]; })) {
    // uniform lengths: written by a kernel, no host-to-device copy
    hipLaunchKernelGGL(k_fill_lengths, dim3(static_cast<unsigned>(std::min<int64_t>((N + 255) / 256, 4096))),
                       dim3(256), 0, ctx->stream, L_dev, N, L[0]);
    EDM_HIP(ctx, hipGetLastError());
  } else {
    // the caller's pageable host array, staged by the runtime
    EDM_HIP(ctx, hipMemcpyAsync(L_dev, L, sizeof(int64_t) * static_cast<size_t>(N), hipMemcpyHostToDevice,
                                ctx->stream));
  }
  for (int E = 1; E <= E_max; ++E) {
    edm::KnnArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.L_dev = L_dev;
    a.E = E;
    a.tau = tau;
    a.Tp = Tp;
    a.k = E + 1;
    a.excl = ctx->excl;
    a.mom = mom;
    a.mom_blocks = mom_blocks;
    a.E_max = E_max;
    a.status = ctx->status;
    EDM_HIP(ctx, edm::launch_knn(a, static_cast<int>(N), L_max, ctx->stream));
  }
  EDM_HIP(ctx, edm::launch_sweep_finalize(mom, mom_blocks, L_dev, N, E_max, tau, Tp, ctx->excl, nullptr,
                                          rho, E_opt, ctx->stream));
  return EDM_OK;
}
