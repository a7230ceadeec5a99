// Host orchestration behind the libedm C ABI (include/edm.h).
//
// Validation happens on the host before anything is enqueued.  Device memory
// beyond the caller's buffers lives in one growable workspace per context;
// small host arrays (lengths, target buckets) travel through a pinned staging
// buffer guarded by an event, so the calls stay asynchronous on the caller's
// stream except where the header says otherwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/edm.h"
#include "kernels.h"
#include "validate.h"

struct edm_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int form = EDM_FORM_PLAIN;
  std::string err;
  char *ws = nullptr;          // device workspace
  size_t ws_bytes = 0;
  int *status = nullptr;       // device status word
  char *pinned = nullptr;      // host staging buffer
  size_t pinned_bytes = 0;
  hipEvent_t pinned_ready = nullptr;  // recorded after the last copy out of `pinned`
  bool pinned_pending = false;
};

namespace {

thread_local std::string g_err;

int set_err(edm_ctx *ctx, int code, const std::string &msg) {
  g_err = msg;
  if (ctx) ctx->err = msg;
  return code;
}

int hip_err(edm_ctx *ctx, hipError_t e, const char *what) {
  return set_err(ctx, EDM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define EDM_HIP(ctx, call)                              \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_err(ctx, e_, #call); \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Upper bound for the workspace (bytes); EDM_WORKSPACE_LIMIT overrides.
size_t workspace_limit() {
  const char *s = std::getenv("EDM_WORKSPACE_LIMIT");
  if (s && *s) {
    const long long v = std::atoll(s);
    if (v > 0) return static_cast<size_t>(v);
  }
  return size_t(8) << 30;
}

// Make sure the workspace holds `bytes`.  Growing it waits for the stream so
// no kernel still uses the old allocation.
int ws_reserve(edm_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return EDM_OK;
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->ws) {
    EDM_HIP(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  const size_t want = align_up(bytes, size_t(1) << 20);
  if (hipMalloc(reinterpret_cast<void **>(&ctx->ws), want) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return set_err(ctx, EDM_E_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  ctx->ws_bytes = want;
  return EDM_OK;
}

// Sub-allocation plan inside the workspace.
struct Plan {
  size_t bytes = 0;
  size_t take(size_t n) {
    const size_t at = align_up(bytes, 256);
    bytes = at + n;
    return at;
  }
};

// Host blob -> device copy through the pinned staging buffer.
int upload(edm_ctx *ctx, const void *host, size_t bytes, void *dev) {
  if (bytes == 0) return EDM_OK;
  if (ctx->pinned_pending) {
    EDM_HIP(ctx, hipEventSynchronize(ctx->pinned_ready));
    ctx->pinned_pending = false;
  }
  if (bytes > ctx->pinned_bytes) {
    if (ctx->pinned) EDM_HIP(ctx, hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    const size_t want = align_up(bytes, size_t(1) << 16);
    if (hipHostMalloc(reinterpret_cast<void **>(&ctx->pinned), want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ctx->pinned = nullptr;
      return set_err(ctx, EDM_E_NOMEM, "pinned staging allocation failed");
    }
    ctx->pinned_bytes = want;
  }
  std::memcpy(ctx->pinned, host, bytes);
  EDM_HIP(ctx, hipMemcpyAsync(dev, ctx->pinned, bytes, hipMemcpyHostToDevice, ctx->stream));
  EDM_HIP(ctx, hipEventRecord(ctx->pinned_ready, ctx->stream));
  ctx->pinned_pending = true;
  return EDM_OK;
}

int check_ctx(edm_ctx *ctx) {
  if (!ctx) return set_err(nullptr, EDM_E_ARG, "NULL context");
  return EDM_OK;
}

#define EDM_RC(expr)            \
  do {                          \
    const int rc_ = (expr);     \
    if (rc_ != EDM_OK) return rc_; \
  } while (0)

}  // namespace

extern "C" {

int edm_ctx_create(edm_ctx **out, void *hip_stream) {
  if (!out) return set_err(nullptr, EDM_E_ARG, "NULL output pointer");
  *out = nullptr;
  edm_ctx *ctx = new (std::nothrow) edm_ctx();
  if (!ctx) return set_err(nullptr, EDM_E_NOMEM, "out of host memory");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&ctx->device);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&ctx->status), sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->pinned_ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    const int rc = hip_err(nullptr, e, "edm_ctx_create");
    if (ctx->status) (void)hipFree(ctx->status);
    if (ctx->pinned_ready) (void)hipEventDestroy(ctx->pinned_ready);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return EDM_OK;
}

int edm_ctx_set_form(edm_ctx *ctx, int form) {
  EDM_RC(check_ctx(ctx));
  if (form != EDM_FORM_PLAIN && form != EDM_FORM_CHOSEN)
    return set_err(ctx, EDM_E_ARG, "unknown form");
  ctx->form = form;
  return EDM_OK;
}

int edm_sync(edm_ctx *ctx) {
  EDM_RC(check_ctx(ctx));
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int flag = 0;
  EDM_HIP(ctx, hipMemcpyAsync(&flag, ctx->status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (flag) {
    EDM_HIP(ctx, hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->stream));
    EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return set_err(ctx, EDM_E_NONFINITE, "a kernel read a non-finite input sample");
  }
  return EDM_OK;
}

const char *edm_last_error(const edm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

void edm_ctx_destroy(edm_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->status) (void)hipFree(ctx->status);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pinned_ready) (void)hipEventDestroy(ctx->pinned_ready);
  delete ctx;
}

int edm_embed(edm_ctx *ctx, const float *x, int64_t L, int32_t E, int32_t tau, float *out) {
  std::string msg;
  const int rc = edm::check_embed(x, L, E, tau, out, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  EDM_HIP(ctx, edm::launch_embed(x, L, E, tau, out, ctx->status, ctx->stream));
  return EDM_OK;
}

int edm_knn(edm_ctx *ctx, const float *x, int64_t L, int32_t E, int32_t tau, int32_t Tp,
            int32_t k, int32_t *idx, float *dist, float *w) {
  std::string msg;
  const int rc = edm::check_knn(x, L, E, tau, Tp, k, idx, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  edm::KnnArgs a{};
  a.X = x;
  a.ldx = L;
  a.L_dev = nullptr;
  a.L_uni = L;
  a.lib_ids = nullptr;
  a.E = E;
  a.tau = tau;
  a.Tp = Tp;
  a.k = k ? k : E + 1;
  a.idx = idx;
  a.dist = dist;
  a.w = w;
  a.tbl_stride = 0;
  a.mom = nullptr;
  a.status = ctx->status;
  EDM_HIP(ctx, edm::launch_knn(a, 1, L, ctx->stream));
  return EDM_OK;
}

int edm_lookup(edm_ctx *ctx, const int32_t *idx, const float *w, int64_t nq, int32_t k, int32_t E,
               int32_t tau, int32_t Tp, const float *Y, int64_t N, int64_t ldy, float *pred,
               float *rho) {
  std::string msg;
  const int rc = edm::check_lookup(idx, w, nq, k, E, tau, Tp, Y, N, ldy, pred, rho, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (N == 0) return EDM_OK;
  edm::LookupArgs b{};
  b.idx = idx;
  b.w = w;
  b.tbl_stride = 0;
  b.lib_ids = nullptr;
  b.Lx_dev = nullptr;
  b.Lx_uni = nq + static_cast<int64_t>(E - 1) * tau + Tp;
  b.E = E;
  b.tau = tau;
  b.Tp = Tp;
  b.k = k;
  b.Y = Y;
  b.ldy = ldy;
  b.Ly_dev = nullptr;
  b.tgt_ids = nullptr;
  b.ntgt = static_cast<int32_t>(N);
  b.rho = rho;
  b.ldrho = 0;
  b.pred = pred;
  b.ldpred = nq;
  b.status = ctx->status;
  EDM_HIP(ctx, edm::launch_lookup(b, 1, nq, ctx->stream));
  return EDM_OK;
}

int edm_simplex_sweep(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N, int64_t ldx,
                      int32_t E_max, int32_t tau, int32_t Tp, float *rho, int32_t *E_opt) {
  std::string msg;
  const int rc = edm::check_sweep(X, L, N, ldx, E_max, tau, Tp, rho, E_opt, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (N == 0) return EDM_OK;
  if (N > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");
  const int64_t L_max = *std::max_element(L, L + N);
  const int32_t mom_blocks = static_cast<int32_t>((L_max + edm::kKnnThreads - 1) / edm::kKnnThreads);
  Plan plan;
  const size_t off_L = plan.take(sizeof(int64_t) * N);
  const size_t off_mom = plan.take(edm::kMomBytes * static_cast<size_t>(N) * E_max * mom_blocks);
  if (plan.bytes > workspace_limit()) return set_err(ctx, EDM_E_NOMEM, "sweep workspace exceeds EDM_WORKSPACE_LIMIT");
  EDM_RC(ws_reserve(ctx, plan.bytes));
  int64_t *L_dev = reinterpret_cast<int64_t *>(ctx->ws + off_L);
  edm::Mom *mom = reinterpret_cast<edm::Mom *>(ctx->ws + off_mom);
  EDM_RC(upload(ctx, L, sizeof(int64_t) * N, L_dev));
  if (ctx->form == EDM_FORM_CHOSEN && tau == 1) {
    // Batched form: one candidate scan per group of E values.
    edm::KnnArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.L_dev = L_dev;
    a.Tp = Tp;
    a.tau = 1;
    a.mom = mom;
    a.mom_blocks = mom_blocks;
    a.E_max = E_max;
    a.status = ctx->status;
    EDM_HIP(ctx, edm::launch_sweep_multi(a, static_cast<int>(N), L_max, ctx->stream));
  } else {
  for (int E = 1; E <= E_max; ++E) {
    edm::KnnArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.L_dev = L_dev;
    a.L_uni = 0;
    a.lib_ids = nullptr;
    a.E = E;
    a.tau = tau;
    a.Tp = Tp;
    a.k = E + 1;
    a.mom = mom;
    a.mom_blocks = mom_blocks;
    a.E_max = E_max;
    a.status = ctx->status;
    EDM_HIP(ctx, edm::launch_knn(a, static_cast<int>(N), L_max, ctx->stream));
  }
  }
  EDM_HIP(ctx, edm::launch_sweep_finalize(mom, mom_blocks, L_dev, N, E_max, tau, Tp, rho, E_opt,
                                          ctx->stream));
  return EDM_OK;
}

int edm_ccm(edm_ctx *ctx, const float *X, const int64_t *Lx, int64_t Nl, int64_t ldx,
            const float *Y, const int64_t *Ly, int64_t Nt, int64_t ldy, const int32_t *E_tgt,
            int32_t tau, int32_t Tp, float *rho) {
  std::string msg;
  const int rc = edm::check_ccm(X, Lx, Nl, ldx, Y, Ly, Nt, ldy, E_tgt, tau, Tp, rho, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (Nl == 0 || Nt == 0) return EDM_OK;
  if (Nl > INT32_MAX || Nt > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");

  // The targets' E decide which tables exist (Section 3.4): read them back.
  std::vector<int32_t> Eh(static_cast<size_t>(Nt));
  EDM_HIP(ctx, hipMemcpyAsync(Eh.data(), E_tgt, sizeof(int32_t) * Nt, hipMemcpyDeviceToHost, ctx->stream));
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<std::vector<int32_t>> bucket(EDM_E_MAX + 1);
  for (int64_t j = 0; j < Nt; ++j) {
    const int e = Eh[static_cast<size_t>(j)];
    if (e < 0 || e > EDM_E_MAX) return set_err(ctx, EDM_E_ARG, "E_tgt outside 0..20");
    if (e > 0) bucket[e].push_back(static_cast<int32_t>(j));
  }

  const int64_t Lx_max = *std::max_element(Lx, Lx + Nl);
  // One blob: Lx, Ly, then every bucket's target ids.
  Plan plan;
  const size_t off_Lx = plan.take(sizeof(int64_t) * Nl);
  const size_t off_Ly = plan.take(sizeof(int64_t) * Nt);
  const size_t off_ids = plan.take(sizeof(int32_t) * Nt);
  const size_t small_bytes = plan.bytes;
  const size_t off_tbl = plan.take(0);
  size_t per_lib_max = 0;  // table bytes of one library at the largest E in use
  for (int e = 1; e <= EDM_E_MAX; ++e) {
    if (bucket[e].empty()) continue;
    const int64_t m = Lx_max - static_cast<int64_t>(e - 1) * tau - Tp;
    if (m > 0) per_lib_max = std::max(per_lib_max, static_cast<size_t>(m) * (e + 1) * 8);
  }
  const size_t limit = workspace_limit();
  if (per_lib_max > 0 && off_tbl + per_lib_max > limit)
    return set_err(ctx, EDM_E_NOMEM, "one library table exceeds EDM_WORKSPACE_LIMIT");
  int64_t batch = Nl;
  if (per_lib_max > 0) batch = std::min<int64_t>(Nl, static_cast<int64_t>((limit - off_tbl) / per_lib_max));
  EDM_RC(ws_reserve(ctx, off_tbl + per_lib_max * static_cast<size_t>(batch) + 256));

  std::vector<char> blob(small_bytes, 0);
  std::memcpy(blob.data() + off_Lx, Lx, sizeof(int64_t) * Nl);
  std::memcpy(blob.data() + off_Ly, Ly, sizeof(int64_t) * Nt);
  std::vector<int64_t> bucket_at(EDM_E_MAX + 1, 0);
  {
    int32_t *ids = reinterpret_cast<int32_t *>(blob.data() + off_ids);
    int64_t at = 0;
    for (int e = 1; e <= EDM_E_MAX; ++e) {
      bucket_at[e] = at;
      for (int32_t j : bucket[e]) ids[at++] = j;
    }
  }
  EDM_RC(upload(ctx, blob.data(), small_bytes, ctx->ws));
  const int64_t *Lx_dev = reinterpret_cast<const int64_t *>(ctx->ws + off_Lx);
  const int64_t *Ly_dev = reinterpret_cast<const int64_t *>(ctx->ws + off_Ly);
  const int32_t *ids_dev = reinterpret_cast<const int32_t *>(ctx->ws + off_ids);

  EDM_HIP(ctx, edm::launch_fill(rho, Nl * Nt, __builtin_nanf(""), ctx->stream));

  for (int e = 1; e <= EDM_E_MAX; ++e) {
    if (bucket[e].empty()) continue;
    const int k = e + 1;
    const int64_t m_max = Lx_max - static_cast<int64_t>(e - 1) * tau - Tp;
    if (m_max - 1 < k) continue;  // no library is long enough for this E
    const int64_t tbl_stride = m_max * k;
    int32_t *tbl_idx = reinterpret_cast<int32_t *>(ctx->ws + off_tbl);
    float *tbl_w = reinterpret_cast<float *>(ctx->ws + off_tbl + sizeof(int32_t) * tbl_stride * batch);
    for (int64_t b0 = 0; b0 < Nl; b0 += batch) {
      const int64_t nb = std::min<int64_t>(batch, Nl - b0);
      const int64_t L_b = *std::max_element(Lx + b0, Lx + b0 + nb);
      edm::KnnArgs a{};
      a.X = X + b0 * ldx;
      a.ldx = ldx;
      a.L_dev = Lx_dev + b0;
      a.lib_ids = nullptr;
      a.E = e;
      a.tau = tau;
      a.Tp = Tp;
      a.k = k;
      a.idx = tbl_idx;
      a.w = tbl_w;
      a.tbl_stride = tbl_stride;
      a.status = ctx->status;
      EDM_HIP(ctx, edm::launch_knn(a, static_cast<int>(nb), L_b, ctx->stream));
      edm::LookupArgs b{};
      b.idx = tbl_idx;
      b.w = tbl_w;
      b.tbl_stride = tbl_stride;
      b.lib_ids = nullptr;
      b.Lx_dev = Lx_dev + b0;
      b.E = e;
      b.tau = tau;
      b.Tp = Tp;
      b.k = k;
      b.Y = Y;
      b.ldy = ldy;
      b.Ly_dev = Ly_dev;
      b.tgt_ids = ids_dev + bucket_at[e];
      b.ntgt = static_cast<int32_t>(bucket[e].size());
      b.rho = rho + b0 * Nt;
      b.ldrho = Nt;
      b.status = ctx->status;
      const int64_t m_b = L_b - static_cast<int64_t>(e - 1) * tau - Tp;
      EDM_HIP(ctx, edm::launch_lookup(b, static_cast<int>(nb), m_b, ctx->stream));
    }
  }
  return EDM_OK;
}

}  // extern "C"
