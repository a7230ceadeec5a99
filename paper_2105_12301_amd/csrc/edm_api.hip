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
#include "ctx.h"
#include "kernels.h"
#include "net_kernels.h"
#include "validate.h"

namespace {
thread_local std::string g_err;
}  // namespace

namespace edm {
namespace host {

int set_err(edm_ctx *ctx, int code, const std::string &msg) {
  g_err = msg;
  if (ctx) ctx->err = msg;
  return code;
}

int hip_err(edm_ctx *ctx, hipError_t e, const char *what) {
  return set_err(ctx, EDM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}


size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Upper bound for the workspace (bytes): half of the current device's
// memory (at least 8 GiB); EDM_WORKSPACE_LIMIT overrides.
size_t workspace_limit() {
  const char *s = std::getenv("EDM_WORKSPACE_LIMIT");
  if (s && *s) {
    const long long v = std::atoll(s);
    if (v > 0) return static_cast<size_t>(v);
  }
  size_t free_b = 0, total_b = 0;
  size_t lim = size_t(8) << 30;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b / 2 > lim) lim = total_b / 2;
  (void)hipGetLastError();
  return lim;
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

// The exact kNN scan of one E for `nslots` libraries: the fused kernel, or in
// EDM_FORM_TWO_KERNEL the paper's distance matrix + row selection, with the
// matrices of up to kTwoKernelPassBytes of libraries per pass in ctx->dmat.
constexpr size_t kTwoKernelPassBytes = size_t(2) << 30;

int knn_exact(edm_ctx *ctx, const edm::KnnArgs &a, int nslots, int64_t L_max) {
  if (ctx->form != EDM_FORM_TWO_KERNEL) {
    EDM_HIP(ctx, edm::launch_knn(a, nslots, L_max, ctx->stream));
    return EDM_OK;
  }
  if (nslots <= 0) return EDM_OK;
  const int64_t m_max = L_max - static_cast<int64_t>(a.E - 1) * a.tau - a.Tp;
  if (m_max < 1) return EDM_OK;
  const int64_t ldd = edm::two_kernel_ld(m_max);
  const size_t per_slot = sizeof(float) * static_cast<size_t>(ldd) * static_cast<size_t>(ldd);
  int per_pass = static_cast<int>(std::max<size_t>(1, std::min<size_t>(kTwoKernelPassBytes / per_slot, nslots)));
  const size_t want = per_slot * static_cast<size_t>(per_pass);
  if (want > workspace_limit())
    return set_err(ctx, EDM_E_NOMEM, "distance matrix exceeds EDM_WORKSPACE_LIMIT");
  if (want > ctx->dmat_bytes) {
    EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->dmat) {
      EDM_HIP(ctx, hipFree(ctx->dmat));
      ctx->dmat = nullptr;
      ctx->dmat_bytes = 0;
    }
    if (hipMalloc(reinterpret_cast<void **>(&ctx->dmat), want) != hipSuccess) {
      (void)hipGetLastError();
      ctx->dmat = nullptr;
      return set_err(ctx, EDM_E_NOMEM, "distance matrix allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->dmat_bytes = want;
  }
  EDM_HIP(ctx, edm::launch_knn_two_kernel(a, nslots, L_max, ctx->dmat, ldd, per_pass, ctx->stream));
  return EDM_OK;
}

namespace {
thread_local edm_ctx *g_timed = nullptr;  // context whose launches are being timed

hipEvent_t take_event(edm_ctx *ctx) {
  if (!ctx->spare_events.empty()) {
    hipEvent_t e = ctx->spare_events.back();
    ctx->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void drop_ranges(edm_ctx *ctx) {
  for (auto &r : ctx->ranges) {
    ctx->spare_events.push_back(r.start);
    ctx->spare_events.push_back(r.stop);
  }
  ctx->ranges.clear();
}
}  // namespace

TimingScope::TimingScope(edm_ctx *ctx) : prev(g_timed) { g_timed = (ctx && ctx->timing) ? ctx : nullptr; }
TimingScope::~TimingScope() { g_timed = prev; }

}  // namespace host

TimedLaunch::TimedLaunch(int fam, hipStream_t s) : family(fam), st(s) {
  edm_ctx *ctx = host::g_timed;
  if (!ctx) return;
  start = host::take_event(ctx);
  if (start && hipEventRecord(start, st) != hipSuccess) {
    (void)hipGetLastError();
    ctx->spare_events.push_back(start);
    start = nullptr;
  }
}

TimedLaunch::~TimedLaunch() {
  edm_ctx *ctx = host::g_timed;
  if (!ctx || !start) return;
  hipEvent_t stop = host::take_event(ctx);
  if (!stop || hipEventRecord(stop, st) != hipSuccess) {
    (void)hipGetLastError();
    ctx->spare_events.push_back(start);
    if (stop) ctx->spare_events.push_back(stop);
    return;
  }
  ctx->ranges.push_back(edm_ctx::TimedRange{family, start, stop});
}

namespace host {


}  // namespace host
}  // namespace edm

using namespace edm::host;


// The batched sweep (tau = 1, no exclusion window) of N contiguous rows: one
// candidate scan per group of E values, through the matrix-core filter for
// E >= 5 in the chosen form, co-moments into mom[N][E_max][mom_blocks].
// plan() reserves the filter's norm buffers (rows in batches of at most
// 1 GiB) in the caller's workspace plan; run() enqueues the scans.
namespace {
struct BatchedSweep {
  bool gram = false;
  int64_t L_max = 0, g_ld = 0, g_batch = 0;
  size_t off_gmu = 0, off_gnrm = 0;

  void plan(const edm_ctx *c, Plan &p, int64_t N, int64_t Lmax, int32_t E_max) {
    L_max = Lmax;
    gram = c->form == EDM_FORM_CHOSEN && E_max >= edm::kGramEMin && L_max <= edm::kGramLMax;
    if (!gram) return;
    g_ld = edm::gram_ld(L_max);
    const size_t g_row = sizeof(uint32_t) * static_cast<size_t>(edm::kGramNE) * g_ld + sizeof(float);
    g_batch = std::max<int64_t>(1, std::min<int64_t>(N, static_cast<int64_t>((size_t(1) << 30) / g_row)));
    off_gmu = p.take(sizeof(float) * g_batch);
    off_gnrm = p.take(sizeof(uint32_t) * static_cast<size_t>(edm::kGramNE) * g_ld * g_batch);
  }

  int run(edm_ctx *c, const float *X, int64_t ldx, const int64_t *L, const int64_t *L_dev, int64_t N,
          int32_t E_max, int32_t Tp, edm::Mom *mom, int32_t mom_blocks) {
    const int64_t step = gram ? g_batch : N;
    for (int64_t b0 = 0; b0 < N; b0 += step) {
      const int64_t nb = std::min<int64_t>(step, N - b0);
      edm::KnnArgs a{};
      a.X = X + b0 * ldx;
      a.ldx = ldx;
      a.L_dev = L_dev + b0;
      a.Tp = Tp;
      a.tau = 1;
      a.mom = reinterpret_cast<edm::Mom *>(reinterpret_cast<char *>(mom) +
                                           edm::kMomBytes * static_cast<size_t>(b0 * E_max) * mom_blocks);
      a.mom_blocks = mom_blocks;
      a.E_max = E_max;
      a.status = c->status;
      int64_t L_b = L_max;
      if (gram) {
        L_b = *std::max_element(L + b0, L + b0 + nb);
        a.gram_mu = reinterpret_cast<float *>(c->ws + off_gmu);
        a.gram_nrm = reinterpret_cast<uint32_t *>(c->ws + off_gnrm);
        a.gram_ld = g_ld;
        EDM_HIP(c, edm::launch_gram_prep(a, static_cast<int>(nb), L_b, c->stream));
      }
      EDM_HIP(c, edm::launch_sweep_multi(a, static_cast<int>(nb), L_b, c->stream));
    }
    return EDM_OK;
  }
};
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
  int rc = e == hipSuccess ? EDM_OK : hip_err(nullptr, e, "edm_ctx_create");
  if (rc == EDM_OK) rc = noalloc_scratch_init(ctx);
  if (rc != EDM_OK) {
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
  if (form != EDM_FORM_PLAIN && form != EDM_FORM_CHOSEN && form != EDM_FORM_BATCHED &&
      form != EDM_FORM_TWO_KERNEL)
    return set_err(ctx, EDM_E_ARG, "unknown form");
  ctx->form = form;
  return EDM_OK;
}

int edm_ctx_set_exclusion_radius(edm_ctx *ctx, int32_t r) {
  EDM_RC(check_ctx(ctx));
  if (r < 0 || r > EDM_L_MAX) return set_err(ctx, EDM_E_ARG, "exclusion radius must be in 0..EDM_L_MAX");
  ctx->excl = r;
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

int edm_ctx_set_timing(edm_ctx *ctx, int on) {
  EDM_RC(check_ctx(ctx));
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  drop_ranges(ctx);
  ctx->timing = on != 0;
  return EDM_OK;
}

int edm_ctx_timing(edm_ctx *ctx, double *ms, int64_t *launches) {
  EDM_RC(check_ctx(ctx));
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (const auto &r : ctx->ranges) {
    float t = 0.0f;
    const hipError_t e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess) {
      drop_ranges(ctx);
      return hip_err(ctx, e, "hipEventElapsedTime");
    }
    if (r.family >= 0 && r.family < EDM_KF_COUNT) {
      if (ms) ms[r.family] += t;
      if (launches) launches[r.family] += 1;
    }
  }
  drop_ranges(ctx);
  return EDM_OK;
}

void edm_ctx_destroy(edm_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  drop_ranges(ctx);
  for (hipEvent_t e : ctx->spare_events) (void)hipEventDestroy(e);
  ctx->spare_events.clear();
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->dmat) (void)hipFree(ctx->dmat);
  if (ctx->status) (void)hipFree(ctx->status);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pinned_ready) (void)hipEventDestroy(ctx->pinned_ready);
  delete ctx;
}

int edm_embed(edm_ctx *ctx, const float *x, int64_t L, int32_t E, int32_t tau, float *out) {
  TimingScope timing_scope(ctx);
  std::string msg;
  const int rc = edm::check_embed(x, L, E, tau, out, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  EDM_HIP(ctx, edm::launch_embed(x, L, E, tau, out, ctx->status, ctx->stream));
  return EDM_OK;
}

int edm_knn(edm_ctx *ctx, const float *x, int64_t L, int32_t E, int32_t tau, int32_t Tp,
            int32_t k, int32_t *idx, float *dist, float *w) {
  TimingScope timing_scope(ctx);
  std::string msg;
  const int rc = edm::check_knn(x, L, E, tau, Tp, k, idx, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (edm::n_query(L, E, tau, Tp) - 1 - 2 * static_cast<int64_t>(ctx->excl) < (k ? k : E + 1))
    return set_err(ctx, EDM_E_SHORT, "series too short for k neighbours outside the exclusion radius");
  if (ctx->form == EDM_FORM_CHOSEN && tau == 1 && (k == 0 || k == E + 1) && dist == nullptr &&
      E >= edm::kGramEMin && L <= edm::kGramLMax && ctx->excl == 0) {
    // Chosen form: the table of one E through the matrix-core filter (the
    // filtered group scan in table mode; the group's other lists stay idle).
    const int64_t nq = L - (E - 1) - Tp;
    const int64_t g_ld = edm::gram_ld(L);
    Plan plan;
    const size_t off_mu = plan.take(sizeof(float));
    const size_t off_nrm = plan.take(sizeof(uint32_t) * static_cast<size_t>(edm::kGramNE) * g_ld);
    const size_t off_w = plan.take(w ? 0 : sizeof(float) * static_cast<size_t>(nq) * (E + 1));
    EDM_RC(ws_reserve(ctx, plan.bytes));
    edm::KnnArgs a{};
    a.X = x;
    a.ldx = L;
    a.L_uni = L;
    a.tau = 1;
    a.Tp = Tp;
    a.E_max = EDM_E_MAX;
    a.status = ctx->status;
    a.need = 1u << (E - 1);
    a.idxE[E] = idx;
    a.wE[E] = w ? w : reinterpret_cast<float *>(ctx->ws + off_w);
    a.strideE[E] = nq * (E + 1);
    a.gram_mu = reinterpret_cast<float *>(ctx->ws + off_mu);
    a.gram_nrm = reinterpret_cast<uint32_t *>(ctx->ws + off_nrm);
    a.gram_ld = g_ld;
    EDM_HIP(ctx, edm::launch_gram_prep(a, 1, L, ctx->stream));
    EDM_HIP(ctx, edm::launch_sweep_multi(a, 1, L, ctx->stream));
    return EDM_OK;
  }
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
  a.excl = ctx->excl;
  a.idx = idx;
  a.dist = dist;
  a.w = w;
  a.tbl_stride = 0;
  a.mom = nullptr;
  a.status = ctx->status;
  return knn_exact(ctx, a, 1, L);
}

int edm_lookup(edm_ctx *ctx, const int32_t *idx, const float *w, int64_t nq, int32_t k, int32_t E,
               int32_t tau, int32_t Tp, const float *Y, int64_t N, int64_t ldy, float *pred,
               float *rho) {
  TimingScope timing_scope(ctx);
  std::string msg;
  const int rc = edm::check_lookup(idx, w, nq, k, E, tau, Tp, Y, N, ldy, pred, rho, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (N == 0) return EDM_OK;
  const int64_t Lx = nq + static_cast<int64_t>(E - 1) * tau + Tp;
  EDM_RC(ws_reserve(ctx, sizeof(float) * static_cast<size_t>(N)));
  float *cm = reinterpret_cast<float *>(ctx->ws);
  EDM_HIP(ctx, edm::launch_target_means(Y, ldy, nullptr, Lx, N, cm, ctx->stream));
  edm::LookupArgs b{};
  b.idx = idx;
  b.w = w;
  b.tbl_stride = 0;
  b.lib_ids = nullptr;
  b.Lx_dev = nullptr;
  b.Lx_uni = Lx;
  b.cmean = cm;
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
  TimingScope timing_scope(ctx);
  std::string msg;
  const int rc = edm::check_sweep(X, L, N, ldx, E_max, tau, Tp, rho, E_opt, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (N == 0) return EDM_OK;
  if (N > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");
  const int64_t L_max = *std::max_element(L, L + N);
  const int32_t mom_blocks = static_cast<int32_t>((L_max + edm::kKnnThreads - 1) / edm::kKnnThreads);
  const bool batched =
      (ctx->form == EDM_FORM_CHOSEN || ctx->form == EDM_FORM_BATCHED) && tau == 1 && ctx->excl == 0;
  Plan plan;
  const size_t off_L = plan.take(sizeof(int64_t) * N);
  const size_t off_mom = plan.take(edm::kMomBytes * static_cast<size_t>(N) * E_max * mom_blocks);
  BatchedSweep bs;
  if (batched) bs.plan(ctx, plan, N, L_max, E_max);
  if (plan.bytes > workspace_limit()) return set_err(ctx, EDM_E_NOMEM, "sweep workspace exceeds EDM_WORKSPACE_LIMIT");
  EDM_RC(ws_reserve(ctx, plan.bytes));
  int64_t *L_dev = reinterpret_cast<int64_t *>(ctx->ws + off_L);
  edm::Mom *mom = reinterpret_cast<edm::Mom *>(ctx->ws + off_mom);
  EDM_RC(upload(ctx, L, sizeof(int64_t) * N, L_dev));
  if (batched) {
    EDM_RC(bs.run(ctx, X, ldx, L, L_dev, N, E_max, Tp, mom, mom_blocks));
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
    a.excl = ctx->excl;
    a.mom = mom;
    a.mom_blocks = mom_blocks;
    a.E_max = E_max;
    a.status = ctx->status;
    EDM_RC(knn_exact(ctx, a, static_cast<int>(N), L_max));
  }
  }
  EDM_HIP(ctx, edm::launch_sweep_finalize(mom, mom_blocks, L_dev, N, E_max, tau, Tp, ctx->excl, nullptr, rho,
                                          E_opt, ctx->stream));
  return EDM_OK;
}

int edm_sweep_ccm(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N, int64_t ldx,
                  int32_t E_max, int32_t tau, float *rho_sweep, int32_t *E_opt, float *rho) {
  TimingScope timing_scope(ctx);
  std::string msg;
  const int rc = edm::check_sweep(X, L, N, ldx, E_max, tau, 1, rho_sweep, E_opt, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  if (N > 0 && !rho) return set_err(ctx, EDM_E_ARG, "NULL rho");
  EDM_RC(check_ctx(ctx));
  if (N == 0) return EDM_OK;
  if (N > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");
  const int64_t L_max = *std::max_element(L, L + N);

  // Workspace of the fused form: the sweep's lists and weights of every E,
  // with one row more per series (query m1 of the cross map): the cross
  // map's tables are these arrays, completed in place.
  const int32_t mom_blocks = static_cast<int32_t>((L_max + edm::kKnnThreads - 1) / edm::kKnnThreads);
  const bool gram = E_max >= edm::kGramEMin && L_max <= edm::kGramLMax;
  const int64_t g_ld = edm::gram_ld(L_max);
  Plan plan;
  const size_t off_L = plan.take(sizeof(int64_t) * N);
  const size_t off_ids = plan.take(sizeof(int32_t) * N);
  const size_t off_at = plan.take(sizeof(int32_t) * (EDM_E_MAX + 2));
  const size_t off_cm = plan.take(sizeof(float) * N);
  const size_t off_mom = plan.take(edm::kMomBytes * static_cast<size_t>(N) * E_max * mom_blocks);
  size_t off_gmu = 0, off_gnrm = 0;
  if (gram) {
    off_gmu = plan.take(sizeof(float) * N);
    off_gnrm = plan.take(sizeof(uint32_t) * static_cast<size_t>(edm::kGramNE) * g_ld * N);
  }
  std::vector<size_t> off_keep(EDM_E_MAX + 1, 0), off_keepw(EDM_E_MAX + 1, 0);
  std::vector<int64_t> keep_stride(EDM_E_MAX + 1, 0);
  for (int E = 1; E <= E_max; ++E) {
    const int64_t m1 = L_max - E;  // sweep queries at E (Tp = 1); the cross map has m1 + 1
    if (m1 > 0) {
      keep_stride[E] = (m1 + 1) * (E + 1);
      off_keep[E] = plan.take(sizeof(int32_t) * static_cast<size_t>(keep_stride[E]) * N);
      off_keepw[E] = plan.take(sizeof(float) * static_cast<size_t>(keep_stride[E]) * N);
    }
  }
  // (the device-memory query only when the workspace must grow)
  bool fused = (ctx->form == EDM_FORM_CHOSEN) && tau == 1 && ctx->excl == 0 &&
               (plan.bytes <= ctx->ws_bytes || plan.bytes <= workspace_limit());
  if (fused && ws_reserve(ctx, plan.bytes) != EDM_OK) fused = false;  // too large to allocate
  if (!fused) {  // the sweep, then the cross map at the selected E (Tp = 0)
    EDM_RC(edm_simplex_sweep(ctx, X, L, N, ldx, E_max, tau, 1, rho_sweep, E_opt));
    return edm_ccm(ctx, X, L, N, ldx, X, L, N, ldx, E_opt, tau, 0, rho);
  }
  int64_t *L_dev = reinterpret_cast<int64_t *>(ctx->ws + off_L);
  int32_t *ids_dev = reinterpret_cast<int32_t *>(ctx->ws + off_ids);
  int32_t *at_dev = reinterpret_cast<int32_t *>(ctx->ws + off_at);
  float *cm_dev = reinterpret_cast<float *>(ctx->ws + off_cm);
  edm::Mom *mom = reinterpret_cast<edm::Mom *>(ctx->ws + off_mom);
  // Equal lengths are written on the device: the call then makes no host
  // transfer and no synchronisation at all (it can be captured in a graph).
  if (std::all_of(L, L + N, [&](int64_t v) { return v == L[0]; }))
    EDM_HIP(ctx, edm::launch_fill_i64(L_dev, N, L[0], ctx->stream));
  else
    EDM_RC(upload(ctx, L, sizeof(int64_t) * N, L_dev));

  edm::KnnArgs a{};
  a.X = X;
  a.ldx = ldx;
  a.L_dev = L_dev;
  a.Tp = 1;
  a.tau = 1;
  a.mom = mom;
  a.mom_blocks = mom_blocks;
  a.E_max = E_max;
  a.status = ctx->status;
  for (int E = 1; E <= E_max; ++E) {
    if (keep_stride[E] == 0) continue;
    a.keepE[E] = reinterpret_cast<int32_t *>(ctx->ws + off_keep[E]);
    a.keepWE[E] = reinterpret_cast<float *>(ctx->ws + off_keepw[E]);
    a.keep_strideE[E] = keep_stride[E];
  }
  if (gram) {
    a.gram_mu = reinterpret_cast<float *>(ctx->ws + off_gmu);
    a.gram_nrm = reinterpret_cast<uint32_t *>(ctx->ws + off_gnrm);
    a.gram_ld = g_ld;
    EDM_HIP(ctx, edm::launch_gram_prep(a, static_cast<int>(N), L_max, ctx->stream));
  }
  EDM_HIP(ctx, edm::launch_sweep_multi(a, static_cast<int>(N), L_max, ctx->stream));
  EDM_HIP(ctx, edm::launch_sweep_finalize(mom, mom_blocks, L_dev, N, E_max, 1, 1, 0, nullptr, rho_sweep,
                                          E_opt, ctx->stream));

  // Targets by their selected E (Section 3.4), grouped on the device: every
  // E is launched, and its kernels exit at once when its bucket is empty.
  EDM_HIP(ctx, edm::launch_group_by_E(E_opt, N, E_max, at_dev, ids_dev, ctx->stream));
  EDM_HIP(ctx, edm::launch_target_means(X, ldx, L_dev, 0, N, cm_dev, ctx->stream));
  EDM_HIP(ctx, edm::launch_fill(rho, N * N, __builtin_nanf(""), ctx->stream));

  for (int e = 1; e <= E_max; ++e) {
    const int64_t m0 = L_max - (e - 1);  // cross-map queries at e (Tp = 0)
    if (m0 - 1 < e + 1) continue;        // no library is long enough for this E
    edm::KnnArgs t{};
    t.X = X;
    t.ldx = ldx;
    t.L_dev = L_dev;
    t.tau = 1;
    t.Tp = 0;
    t.E_max = EDM_E_MAX;
    t.status = ctx->status;
    t.need = 1u << (e - 1);
    t.keepE[e] = a.keepE[e];
    t.keepWE[e] = a.keepWE[e];
    t.keep_strideE[e] = a.keep_strideE[e];
    t.group_at = at_dev;
    const int64_t stride = a.keep_strideE[e];  // m0 * (e + 1): the kept arrays are the tables
    t.idxE[e] = a.keepE[e];
    t.wE[e] = a.keepWE[e];
    t.strideE[e] = stride;
    EDM_HIP(ctx, edm::launch_tables_from_sweep(t, e, static_cast<int>(N), L_max, ctx->stream));
    edm::LookupArgs b{};
    b.idx = t.idxE[e];
    b.w = t.wE[e];
    b.tbl_stride = stride;
    b.Lx_dev = L_dev;
    b.E = e;
    b.tau = 1;
    b.Tp = 0;
    b.k = e + 1;
    b.Y = X;
    b.cmean = cm_dev;
    b.ldy = ldx;
    b.Ly_dev = L_dev;
    b.bucket_ids = ids_dev;
    b.bucket_at = at_dev;
    b.rho = rho;
    b.ldrho = N;
    b.status = ctx->status;
    EDM_HIP(ctx, edm::launch_lookup_bucket(b, static_cast<int>(N), m0, N, ctx->stream));
  }
  return EDM_OK;
}

int edm_ccm(edm_ctx *ctx, const float *X, const int64_t *Lx, int64_t Nl, int64_t ldx,
            const float *Y, const int64_t *Ly, int64_t Nt, int64_t ldy, const int32_t *E_tgt,
            int32_t tau, int32_t Tp, float *rho) {
  TimingScope timing_scope(ctx);
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
  const size_t off_cm = plan.take(sizeof(float) * Nt);
  const size_t off_tbl = plan.take(0);
  // Table bytes of one library: the largest E in use (plain form, one E at a
  // time) or every E in use together (chosen form, one scan per E group).
  const bool batched =
      (ctx->form == EDM_FORM_CHOSEN || ctx->form == EDM_FORM_BATCHED) && tau == 1 && ctx->excl == 0;
  const bool gram = batched && ctx->form == EDM_FORM_CHOSEN && Lx_max <= edm::kGramLMax;
  const int64_t g_ld = edm::gram_ld(Lx_max);
  // Filter norms and centring constant of one library (chosen form).
  const size_t per_lib_gram =
      gram ? align_up(sizeof(uint32_t) * static_cast<size_t>(edm::kGramNE) * g_ld + sizeof(float), 256) : 0;
  size_t per_lib_max = 0;
  std::vector<size_t> off_E(EDM_E_MAX + 1, 0);
  for (int e = 1; e <= EDM_E_MAX; ++e) {
    if (bucket[e].empty()) continue;
    const int64_t m = Lx_max - static_cast<int64_t>(e - 1) * tau - Tp;
    if (m <= 0) continue;
    const size_t b = align_up(static_cast<size_t>(m) * (e + 1) * 8, 256);
    if (batched) {
      off_E[e] = per_lib_max;
      per_lib_max += b;
    } else {
      per_lib_max = std::max(per_lib_max, b);
    }
  }
  const size_t limit = workspace_limit();
  if (per_lib_max > 0 && off_tbl + per_lib_max + per_lib_gram > limit)
    return set_err(ctx, EDM_E_NOMEM, "one library table exceeds EDM_WORKSPACE_LIMIT");
  int64_t batch = Nl;
  if (per_lib_max > 0)
    batch = std::min<int64_t>(Nl, static_cast<int64_t>((limit - off_tbl) / (per_lib_max + per_lib_gram)));
  const size_t off_g = off_tbl + per_lib_max * static_cast<size_t>(batch);
  EDM_RC(ws_reserve(ctx, off_g + per_lib_gram * static_cast<size_t>(batch) + 256));

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
  float *cm_dev = reinterpret_cast<float *>(ctx->ws + off_cm);
  const int32_t *ids_dev = reinterpret_cast<const int32_t *>(ctx->ws + off_ids);

  EDM_HIP(ctx, edm::launch_fill(rho, Nl * Nt, __builtin_nanf(""), ctx->stream));
  EDM_HIP(ctx, edm::launch_target_means(Y, ldy, Ly_dev, 0, Nt, cm_dev, ctx->stream));

  if (batched) {
    // Chosen form: per library batch, one scan per E group writes the tables
    // of every E in use, then one lookup launch per E.
    uint32_t need = 0;
    for (int e = 1; e <= EDM_E_MAX; ++e) {
      const int64_t m_max = Lx_max - static_cast<int64_t>(e - 1) - Tp;
      if (!bucket[e].empty() && m_max - 1 >= e + 1) need |= 1u << (e - 1);
    }
    for (int64_t b0 = 0; b0 < Nl && need; b0 += batch) {
      const int64_t nb = std::min<int64_t>(batch, Nl - b0);
      const int64_t L_b = *std::max_element(Lx + b0, Lx + b0 + nb);
      edm::KnnArgs a{};
      a.X = X + b0 * ldx;
      a.ldx = ldx;
      a.L_dev = Lx_dev + b0;
      a.tau = 1;
      a.Tp = Tp;
      a.E_max = EDM_E_MAX;
      a.status = ctx->status;
      a.need = need;
      for (int e = 1; e <= EDM_E_MAX; ++e) {
        if (!((need >> (e - 1)) & 1u)) continue;
        const int64_t m_max = Lx_max - static_cast<int64_t>(e - 1) - Tp;
        const int64_t stride = m_max * (e + 1);
        char *base = ctx->ws + off_tbl + off_E[e] * static_cast<size_t>(batch);
        a.idxE[e] = reinterpret_cast<int32_t *>(base);
        a.wE[e] = reinterpret_cast<float *>(base + sizeof(int32_t) * stride * batch);
        a.strideE[e] = stride;
      }
      bool gram_b = false;
      for (int e = edm::kGramEMin; e <= EDM_E_MAX; ++e) gram_b |= gram && ((need >> (e - 1)) & 1u);
      if (gram_b) {
        a.gram_mu = reinterpret_cast<float *>(ctx->ws + off_g);
        a.gram_nrm = reinterpret_cast<uint32_t *>(ctx->ws + align_up(off_g + sizeof(float) * batch, 256));
        a.gram_ld = g_ld;
        EDM_HIP(ctx, edm::launch_gram_prep(a, static_cast<int>(nb), L_b, ctx->stream));
      }
      EDM_HIP(ctx, edm::launch_sweep_multi(a, static_cast<int>(nb), L_b, ctx->stream));
      for (int e = 1; e <= EDM_E_MAX; ++e) {
        if (!((need >> (e - 1)) & 1u)) continue;
        edm::LookupArgs b{};
        b.idx = a.idxE[e];
        b.w = a.wE[e];
        b.tbl_stride = a.strideE[e];
        b.Lx_dev = Lx_dev + b0;
        b.E = e;
        b.tau = 1;
        b.Tp = Tp;
        b.k = e + 1;
        b.Y = Y;
        b.cmean = cm_dev;
        b.ldy = ldy;
        b.Ly_dev = Ly_dev;
        b.tgt_ids = ids_dev + bucket_at[e];
        b.ntgt = static_cast<int32_t>(bucket[e].size());
        b.rho = rho + b0 * Nt;
        b.ldrho = Nt;
        b.status = ctx->status;
        const int64_t m_b = L_b - static_cast<int64_t>(e - 1) - Tp;
        EDM_HIP(ctx, edm::launch_lookup(b, static_cast<int>(nb), m_b, ctx->stream));
      }
    }
    return EDM_OK;
  }

  for (int e = 1; e <= EDM_E_MAX; ++e) {
    if (bucket[e].empty()) continue;
    const int k = e + 1;
    const int64_t m_max = Lx_max - static_cast<int64_t>(e - 1) * tau - Tp;
    if (m_max - 1 - 2 * static_cast<int64_t>(ctx->excl) < k) continue;  // no library is long enough
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
      a.excl = ctx->excl;
      a.idx = tbl_idx;
      a.w = tbl_w;
      a.tbl_stride = tbl_stride;
      a.status = ctx->status;
      EDM_RC(knn_exact(ctx, a, static_cast<int>(nb), L_b));
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
      b.excl = ctx->excl;
      b.Y = Y;
      b.cmean = cm_dev;
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

int edm_ccm_subsample(edm_ctx *ctx, const float *x, int64_t L, const float *Y, int64_t Nt,
                      int64_t ldy, int32_t E, int32_t tau, int32_t Tp, const int32_t *sets,
                      const int64_t *set_off, int64_t S, int32_t *idx, float *rho) {
  TimingScope timing_scope(ctx);
  std::string msg;
  if (!x) return set_err(ctx, EDM_E_ARG, "NULL library");
  if (E > EDM_E_MAX) return set_err(ctx, EDM_E_ARG, "E must be <= 20");
  const int rc = edm::check_embedding(L, E, tau, Tp, E + 1, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  EDM_RC(check_ctx(ctx));
  if (S < 0 || Nt < 0) return set_err(ctx, EDM_E_ARG, "S and Nt must be >= 0");
  if (S > 0 && (!sets || !set_off)) return set_err(ctx, EDM_E_ARG, "NULL subsample sets");
  if (S > 0 && Nt > 0 && (!Y || !rho)) return set_err(ctx, EDM_E_ARG, "NULL pointer (Y and rho)");
  if (Nt > 0 && ldy < L) return set_err(ctx, EDM_E_ARG, "ldy shorter than the library");
  if (S > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many subsamples");
  const int64_t m = edm::n_query(L, E, tau, Tp);
  const int K = E + 1;
  if (S > 0 && set_off[0] != 0) return set_err(ctx, EDM_E_ARG, "set_off[0] must be 0");
  for (int64_t s = 0; s < S; ++s) {
    const int64_t b0 = set_off[s], b1 = set_off[s + 1];
    if (b1 < b0) return set_err(ctx, EDM_E_ARG, "set_off must be non-decreasing");
    if (b1 - b0 - (2 * static_cast<int64_t>(ctx->excl) + 1) < K)
      return set_err(ctx, EDM_E_SHORT, "subsample too small for k neighbours outside the exclusion radius");
    for (int64_t i = b0; i < b1; ++i) {
      if (sets[i] < 0 || sets[i] >= m) return set_err(ctx, EDM_E_ARG, "subsample index outside [0, nq)");
      if (i > b0 && sets[i] <= sets[i - 1]) return set_err(ctx, EDM_E_ARG, "subsample indices must ascend strictly");
    }
  }
  if (S == 0) return EDM_OK;
  const int64_t n_idx = set_off[S];
  const int64_t stride = m * K;
  Plan plan;
  const size_t off_sets = plan.take(sizeof(int32_t) * static_cast<size_t>(n_idx));
  const size_t off_off = plan.take(sizeof(int64_t) * static_cast<size_t>(S + 1));
  const size_t small = plan.bytes;
  const size_t off_idx = plan.take(idx ? 0 : sizeof(int32_t) * static_cast<size_t>(stride) * S);
  const size_t off_cm = plan.take(sizeof(float) * static_cast<size_t>(Nt));
  const size_t off_w = plan.take(sizeof(float) * static_cast<size_t>(stride) * S);
  if (plan.bytes > workspace_limit()) return set_err(ctx, EDM_E_NOMEM, "subsample tables exceed EDM_WORKSPACE_LIMIT");
  EDM_RC(ws_reserve(ctx, plan.bytes));
  std::vector<char> blob(small, 0);
  std::memcpy(blob.data() + off_sets, sets, sizeof(int32_t) * static_cast<size_t>(n_idx));
  std::memcpy(blob.data() + off_off, set_off, sizeof(int64_t) * static_cast<size_t>(S + 1));
  EDM_RC(upload(ctx, blob.data(), small, ctx->ws));
  edm::KnnArgs a{};
  a.X = x;
  a.ldx = L;
  a.L_uni = L;
  a.E = E;
  a.tau = tau;
  a.Tp = Tp;
  a.k = K;
  a.excl = ctx->excl;
  a.idx = idx ? idx : reinterpret_cast<int32_t *>(ctx->ws + off_idx);
  a.w = reinterpret_cast<float *>(ctx->ws + off_w);
  a.tbl_stride = stride;
  a.status = ctx->status;
  EDM_HIP(ctx, edm::launch_knn_subsets(a, reinterpret_cast<const int32_t *>(ctx->ws + off_sets),
                                       reinterpret_cast<const int64_t *>(ctx->ws + off_off),
                                       static_cast<int>(S), ctx->stream));
  if (Nt == 0) return EDM_OK;
  float *cm = reinterpret_cast<float *>(ctx->ws + off_cm);
  EDM_HIP(ctx, edm::launch_target_means(Y, ldy, nullptr, L, Nt, cm, ctx->stream));
  edm::LookupArgs b{};
  b.idx = a.idx;
  b.w = a.w;
  b.tbl_stride = stride;
  b.Lx_uni = L;
  b.cmean = cm;
  b.E = E;
  b.tau = tau;
  b.Tp = Tp;
  b.k = K;
  b.Y = Y;
  b.ldy = ldy;
  b.ntgt = static_cast<int32_t>(Nt);
  b.rho = rho;
  b.ldrho = Nt;
  b.status = ctx->status;
  EDM_HIP(ctx, edm::launch_lookup(b, static_cast<int>(S), m, ctx->stream));
  return EDM_OK;
}

int64_t edm_net_param_count(int32_t C) {
  if (C < 1 || C > EDM_NET_C_MAX) return -1;
  return edm::net_param_count(C);
}

namespace {
int check_net(edm_ctx *ctx, const void *params, int32_t C, const void *X, int64_t B, int64_t L,
              int64_t ldx) {
  if (!params || (B > 0 && !X)) return set_err(ctx, EDM_E_ARG, "NULL pointer");
  if (C < 1 || C > EDM_NET_C_MAX) return set_err(ctx, EDM_E_ARG, "C must be in 1..64");
  if (B < 0 || L < 1 || ldx < L) return set_err(ctx, EDM_E_ARG, "need B >= 0, L >= 1, ldx >= L");
  if (B > 65535) return set_err(ctx, EDM_E_ARG, "at most 65535 series per call");
  return EDM_OK;
}

int net_ws(edm_ctx *ctx, int32_t C, int64_t B, int64_t L) {
  const size_t bytes = sizeof(float) * static_cast<size_t>(edm::net_workspace_floats(C, B, L));
  if (bytes > workspace_limit()) return set_err(ctx, EDM_E_NOMEM, "network workspace exceeds EDM_WORKSPACE_LIMIT: use smaller batches");
  return ws_reserve(ctx, bytes);
}
}  // namespace

int edm_net_forward(edm_ctx *ctx, const float *params, int32_t C, const float *X, int64_t B,
                    int64_t L, int64_t ldx, float *logits) {
  TimingScope timing_scope(ctx);
  EDM_RC(check_net(ctx, params, C, X, B, L, ldx));
  if (B > 0 && !logits) return set_err(ctx, EDM_E_ARG, "NULL logits");
  EDM_RC(check_ctx(ctx));
  if (B == 0) return EDM_OK;
  EDM_RC(net_ws(ctx, C, B, L));
  EDM_HIP(ctx, edm::net_forward(params, C, X, B, L, ldx, reinterpret_cast<float *>(ctx->ws), logits, ctx->stream));
  return EDM_OK;
}

int edm_net_forward_bf16(edm_ctx *ctx, const float *params, int32_t C, const float *X, int64_t B,
                         int64_t L, int64_t ldx, float *logits) {
  TimingScope timing_scope(ctx);
  EDM_RC(check_net(ctx, params, C, X, B, L, ldx));
  if (C != 32 && C != 64) return set_err(ctx, EDM_E_ARG, "the BF16 forward needs C = 32 or 64");
  if (B > 0 && !logits) return set_err(ctx, EDM_E_ARG, "NULL logits");
  EDM_RC(check_ctx(ctx));
  if (B == 0) return EDM_OK;
  EDM_RC(net_ws(ctx, C, B, L));
  EDM_HIP(ctx, edm::net_forward_bf16(params, C, X, B, L, ldx, reinterpret_cast<float *>(ctx->ws), logits, ctx->stream));
  return EDM_OK;
}

int edm_net_loss_grad(edm_ctx *ctx, const float *params, int32_t C, const float *X,
                      const int32_t *labels, int64_t B, int64_t L, int64_t ldx, float *loss,
                      float *grad) {
  TimingScope timing_scope(ctx);
  EDM_RC(check_net(ctx, params, C, X, B, L, ldx));
  if (B < 1 || !labels || !loss || !grad) return set_err(ctx, EDM_E_ARG, "need B >= 1 and labels, loss, grad");
  EDM_RC(check_ctx(ctx));
  EDM_RC(net_ws(ctx, C, B, L));
  EDM_HIP(ctx, edm::net_loss_grad(params, C, X, labels, B, L, ldx, reinterpret_cast<float *>(ctx->ws), loss, grad, ctx->stream));
  return EDM_OK;
}

int edm_net_adam(edm_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n,
                 int32_t step, float lr, float beta1, float beta2, float eps) {
  TimingScope timing_scope(ctx);
  if (!params || !grad || !m || !v) return set_err(ctx, EDM_E_ARG, "NULL pointer");
  if (n < 0 || step < 1) return set_err(ctx, EDM_E_ARG, "need n >= 0 and step >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return set_err(ctx, EDM_E_ARG, "need 0 <= beta < 1 and eps >= 0");
  EDM_RC(check_ctx(ctx));
  if (n == 0) return EDM_OK;
  EDM_HIP(ctx, edm::net_adam(params, grad, m, v, n, step, lr, beta1, beta2, eps, ctx->stream));
  return EDM_OK;
}

int edm_select_E(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N, int64_t ldx,
                 int32_t E_max, int32_t tau, int32_t Tp, const float *logits, int32_t m_top,
                 float min_conf, float *rho, int32_t *E_opt, int64_t *n_fallback) {
  TimingScope timing_scope(ctx);
  std::string msg;
  const int rc = edm::check_sweep(X, L, N, ldx, E_max, tau, Tp, rho, E_opt, msg);
  if (rc != EDM_OK) return set_err(ctx, rc, msg);
  if (N > 0 && !logits) return set_err(ctx, EDM_E_ARG, "NULL logits");
  if (m_top < 1 || m_top > EDM_NET_CLASSES) return set_err(ctx, EDM_E_ARG, "m_top must be in 1..20");
  if (!(min_conf >= 0.0f && min_conf <= 1.0f)) return set_err(ctx, EDM_E_ARG, "min_conf must be in [0, 1]");
  EDM_RC(check_ctx(ctx));
  if (n_fallback) *n_fallback = 0;
  if (N == 0) return EDM_OK;
  if (N > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");
  const int64_t L_max = *std::max_element(L, L + N);
  const int32_t mom_blocks = static_cast<int32_t>((L_max + edm::kKnnThreads - 1) / edm::kKnnThreads);
  const bool batched =
      (ctx->form == EDM_FORM_CHOSEN || ctx->form == EDM_FORM_BATCHED) && tau == 1 && ctx->excl == 0;
  const size_t mom_row = edm::kMomBytes * static_cast<size_t>(E_max) * mom_blocks;
  Plan plan;
  const size_t off_L = plan.take(sizeof(int64_t) * N);
  const size_t off_ids = plan.take(sizeof(int32_t) * static_cast<size_t>(N) * (E_max + 1));
  const size_t off_cand = plan.take(sizeof(uint32_t) * N);
  const size_t off_mom = plan.take(mom_row * N);
  if (plan.bytes > workspace_limit()) return set_err(ctx, EDM_E_NOMEM, "selection workspace exceeds EDM_WORKSPACE_LIMIT");
  EDM_RC(ws_reserve(ctx, plan.bytes));
  EDM_RC(upload(ctx, L, sizeof(int64_t) * N, ctx->ws + off_L));
  EDM_HIP(ctx, edm::launch_candidates(logits, N, E_max, m_top, min_conf,
                                      reinterpret_cast<uint32_t *>(ctx->ws + off_cand), ctx->stream));
  std::vector<uint32_t> ch(static_cast<size_t>(N));
  EDM_HIP(ctx, hipMemcpyAsync(ch.data(), ctx->ws + off_cand, sizeof(uint32_t) * N, hipMemcpyDeviceToHost,
                              ctx->stream));
  EDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const uint32_t all = (E_max >= 32) ? 0xffffffffu : ((1u << E_max) - 1u);
  int64_t fb = 0;
  for (int64_t s = 0; s < N; ++s) fb += (ch[static_cast<size_t>(s)] == all && m_top < E_max);
  // In the batched forms a series with every E to evaluate (the fallback)
  // takes the batched sweep: its rows are packed, swept, and their
  // co-moments scattered back.  The others run one exact scan per proposed E.
  std::vector<int32_t> full;
  if (batched)
    for (int64_t s = 0; s < N; ++s)
      if (ch[static_cast<size_t>(s)] == all) full.push_back(static_cast<int32_t>(s));
  const int64_t n_full = static_cast<int64_t>(full.size());
  std::vector<int32_t> ids(full);
  std::vector<int64_t> at(E_max + 2, 0);
  for (int E = 1; E <= E_max; ++E) {
    at[E] = static_cast<int64_t>(ids.size());
    for (int64_t s = 0; s < N; ++s) {
      const uint32_t c = ch[static_cast<size_t>(s)];
      const int64_t m = L[s] - static_cast<int64_t>(E - 1) * tau - Tp;
      if (((c >> (E - 1)) & 1u) && !(batched && c == all) && m - 1 - 2 * ctx->excl >= E + 1)
        ids.push_back(static_cast<int32_t>(s));
    }
  }
  at[E_max + 1] = static_cast<int64_t>(ids.size());
  // the packed rows of the fallback series, their lengths and co-moments
  BatchedSweep bs;
  size_t off_X = 0, off_Lf = 0, off_momf = 0;
  std::vector<int64_t> Lf(static_cast<size_t>(n_full));
  for (int64_t i = 0; i < n_full; ++i) Lf[static_cast<size_t>(i)] = L[full[static_cast<size_t>(i)]];
  if (n_full > 0) {
    off_X = plan.take(sizeof(float) * static_cast<size_t>(L_max) * n_full);
    off_Lf = plan.take(sizeof(int64_t) * n_full);
    off_momf = plan.take(mom_row * n_full);
    bs.plan(ctx, plan, n_full, L_max, E_max);
    if (plan.bytes > workspace_limit())
      return set_err(ctx, EDM_E_NOMEM, "selection workspace exceeds EDM_WORKSPACE_LIMIT");
    // a larger workspace is a new allocation (the stream is idle): the
    // lengths and candidate sets go up again
    const bool moved = plan.bytes > ctx->ws_bytes;
    EDM_RC(ws_reserve(ctx, plan.bytes));
    if (moved) {
      EDM_RC(upload(ctx, L, sizeof(int64_t) * N, ctx->ws + off_L));
      EDM_RC(upload(ctx, ch.data(), sizeof(uint32_t) * N, ctx->ws + off_cand));
    }
  }
  int64_t *L_dev = reinterpret_cast<int64_t *>(ctx->ws + off_L);
  int32_t *ids_dev = reinterpret_cast<int32_t *>(ctx->ws + off_ids);
  const uint32_t *cand = reinterpret_cast<const uint32_t *>(ctx->ws + off_cand);
  edm::Mom *mom = reinterpret_cast<edm::Mom *>(ctx->ws + off_mom);
  if (!ids.empty()) EDM_RC(upload(ctx, ids.data(), sizeof(int32_t) * ids.size(), ids_dev));
  if (n_full > 0) {
    float *Xf = reinterpret_cast<float *>(ctx->ws + off_X);
    int64_t *Lf_dev = reinterpret_cast<int64_t *>(ctx->ws + off_Lf);
    edm::Mom *momf = reinterpret_cast<edm::Mom *>(ctx->ws + off_momf);
    EDM_RC(upload(ctx, Lf.data(), sizeof(int64_t) * n_full, Lf_dev));
    EDM_HIP(ctx, edm::launch_copy_rows(X, ldx, Xf, L_max, ids_dev, n_full, L_max, false, ctx->stream));
    EDM_RC(bs.run(ctx, Xf, L_max, Lf.data(), Lf_dev, n_full, E_max, Tp, momf, mom_blocks));
    const int64_t mw = static_cast<int64_t>(mom_row / sizeof(uint32_t));
    EDM_HIP(ctx, edm::launch_copy_rows(momf, mw, mom, mw, ids_dev, n_full, mw, true, ctx->stream));
  }
  for (int E = 1; E <= E_max; ++E) {
    const int64_t n_E = at[E + 1] - at[E];
    if (n_E == 0) continue;
    edm::KnnArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.L_dev = L_dev;
    a.lib_ids = ids_dev + at[E];
    a.E = E;
    a.tau = tau;
    a.Tp = Tp;
    a.k = E + 1;
    a.excl = ctx->excl;
    a.mom = mom;
    a.mom_blocks = mom_blocks;
    a.E_max = E_max;
    a.status = ctx->status;
    EDM_RC(knn_exact(ctx, a, static_cast<int>(n_E), L_max));
  }
  EDM_HIP(ctx, edm::launch_sweep_finalize(mom, mom_blocks, L_dev, N, E_max, tau, Tp, ctx->excl, cand, rho, E_opt,
                                          ctx->stream));
  if (n_fallback) *n_fallback = fb;
  return EDM_OK;
}

}  // extern "C"
