// Batched CCM plan (include/edm.h, edm_ccm_plan_*): libraries of uneven
// length and targets of uneven E as work lists for persistent kernels,
// captured once into a HIP graph and replayed.
//
// Grouping follows the paper's Section 3.4: targets are bucketed by their
// optimal E and each library's table for an E is built once and reused by
// every target of that E.  Beyond the paper: tables of all E a library needs
// come from one candidate scan per E group; libraries are processed longest
// first; inside each E bucket the targets are sorted by length (longest
// first), so the targets a library may cross-map (L_target >= L_library) are
// a prefix of the bucket and no lookup work is spent on undefined pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/edm.h"
#include "ctx.h"
#include "kernels.h"

using namespace edm::host;

namespace {

// Table work lists: the exact E groups (lists 0-4), the exact E 1-4 below
// the filter (list 5), and the matrix-core filtered groups of the chosen form
// (lists 6-11, kGramGroups).  A library up to kGramLMax samples in the chosen
// form takes lists 5-11, any other library lists 0-4.
constexpr int kNGroups = 5;
constexpr int kGroupLo[kNGroups] = {1, 9, 13, 16, 19};
constexpr int kGroupHi[kNGroups] = {8, 12, 15, 18, 20};
constexpr int kNGram = 6;
// filtered lists come twice: series whose samples fit in LDS, then longer ones
constexpr int kNLists = kNGroups + 1 + 2 * kNGram;

struct Batch {
  int64_t L_max = 0, Lg_max = 0, Ls_max = 0;  // longest library; longest filtered; longest short filtered
  std::array<int64_t, kNLists> t_begin{}, t_count{};
  std::array<int64_t, EDM_E_MAX + 1> l_begin{}, l_count{}, lds_floats{};
};

// E range and eligibility of table list c for a library (filtered or not;
// long: more samples than fit in LDS next to the filter's arrays).
inline bool list_range(int c, bool filt, bool long_, int &lo, int &hi) {
  if (c < kNGroups) {
    lo = kGroupLo[c];
    hi = kGroupHi[c];
    return !filt;
  }
  if (c == kNGroups) {
    lo = 1;
    hi = edm::kGramEMin - 1;
    return filt;
  }
  const int f = (c - kNGroups - 1) % kNGram;
  const bool want_long = c - kNGroups - 1 >= kNGram;
  lo = edm::kGramGroups[f][0];
  hi = edm::kGramGroups[f][1];
  return filt && long_ == want_long;
}

}  // namespace

struct edm_plan {
  int64_t Nl = 0, Nt = 0, ldx = 0, ldy = 0;
  int Tp = 0;
  edm_tune tune{};
  int n_cu = 0;
  char *dev = nullptr;  // one device allocation for everything below
  int64_t *Lx_dev = nullptr, *Ly_dev = nullptr, *tbl_off = nullptr;
  uint32_t *need = nullptr;
  int32_t *bucket_ids = nullptr, *bucket_at = nullptr;
  int *counters = nullptr;
  int n_counters = 0;
  int32_t *tbl_idx = nullptr;
  float *tbl_w = nullptr;
  edm::TableItem *titems = nullptr;
  edm::LookupItem *litems = nullptr;
  int32_t *item_libs = nullptr;
  bool filtered = false;  // some library runs through the matrix-core filter
  int64_t Lg_max = 0, gram_ld = 0;
  float *gram_mu = nullptr;
  uint32_t *gram_nrm = nullptr;
  float *cmean = nullptr;  // targets' centring constants (computed in every run)
  std::vector<Batch> batches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const float *gX = nullptr, *gY = nullptr;
  float *grho = nullptr;
  hipStream_t gstream = nullptr;
};

extern "C" {

void edm_tune_default(edm_tune *t) {
  if (!t) return;
  t->tables_wg_per_cu = 0;
  t->lookup_wg_per_cu = 0;
  t->lookup_targets = 16;
  t->filter_stride = 0;
}

void edm_ccm_plan_destroy(edm_ctx *ctx, edm_plan *plan) {
  if (!plan) return;
  if (ctx) (void)hipStreamSynchronize(ctx->stream);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->dev) (void)hipFree(plan->dev);
  delete plan;
}

int edm_ccm_plan_create(edm_ctx *ctx, const int64_t *Lx, int64_t Nl, int64_t ldx,
                        const int64_t *Ly, int64_t Nt, int64_t ldy, const int32_t *E_tgt,
                        int32_t Tp, const edm_tune *tune, edm_plan **out) {
  if (!out) return set_err(ctx, EDM_E_ARG, "NULL plan pointer");
  *out = nullptr;
  if (Nl < 1 || Nt < 1 || !Lx || !Ly || !E_tgt) return set_err(ctx, EDM_E_ARG, "need Nl, Nt >= 1 and host Lx, Ly, E_tgt");
  if (Nl > INT32_MAX || Nt > INT32_MAX) return set_err(ctx, EDM_E_ARG, "too many series");
  if (Tp < 0) return set_err(ctx, EDM_E_ARG, "Tp must be >= 0");
  for (int64_t i = 0; i < Nl; ++i)
    if (Lx[i] < 1 || Lx[i] > ldx || Lx[i] > EDM_L_MAX) return set_err(ctx, EDM_E_ARG, "library length outside 1..min(ldx, EDM_L_MAX)");
  for (int64_t j = 0; j < Nt; ++j) {
    if (Ly[j] < 1 || Ly[j] > ldy || Ly[j] > EDM_L_MAX) return set_err(ctx, EDM_E_ARG, "target length outside 1..min(ldy, EDM_L_MAX)");
    if (E_tgt[j] < 0 || E_tgt[j] > EDM_E_MAX) return set_err(ctx, EDM_E_ARG, "E_tgt outside 0..20");
  }
  edm_tune tn;
  edm_tune_default(&tn);
  if (tune) tn = *tune;
  if (tn.tables_wg_per_cu < 0 || tn.tables_wg_per_cu > 8 || tn.lookup_wg_per_cu < 0 ||
      tn.lookup_wg_per_cu > 16 || tn.lookup_targets < 1 || tn.lookup_targets > edm::kLookupItemMaxTargets ||
      tn.filter_stride < 0 || tn.filter_stride > 8)
    return set_err(ctx, EDM_E_ARG, "tune out of range");
  EDM_RC(check_ctx(ctx));
  if (ctx->excl != 0) return set_err(ctx, EDM_E_ARG, "batched plans need exclusion radius 0");

  edm_plan *P = new (std::nothrow) edm_plan();
  if (!P) return set_err(ctx, EDM_E_NOMEM, "out of host memory");
  P->Nl = Nl;
  P->Nt = Nt;
  P->ldx = ldx;
  P->ldy = ldy;
  P->Tp = Tp;
  P->tune = tn;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || n_cu < 1) n_cu = 256;
  P->n_cu = n_cu;

  // Targets by E, each bucket sorted by length (longest first, then index).
  std::vector<std::vector<int32_t>> bucket(EDM_E_MAX + 1);
  for (int64_t j = 0; j < Nt; ++j)
    if (E_tgt[j] > 0) bucket[E_tgt[j]].push_back(static_cast<int32_t>(j));
  for (auto &b : bucket)
    std::stable_sort(b.begin(), b.end(), [&](int32_t u, int32_t v) { return Ly[u] > Ly[v]; });
  std::vector<int32_t> ids;
  std::vector<int32_t> at(EDM_E_MAX + 2, 0);
  for (int e = 0; e <= EDM_E_MAX; ++e) {
    at[e] = static_cast<int32_t>(ids.size());
    if (e > 0) ids.insert(ids.end(), bucket[e].begin(), bucket[e].end());
  }
  at[EDM_E_MAX + 1] = static_cast<int32_t>(ids.size());
  // number of targets of bucket E with length >= L (a prefix of the bucket)
  auto defined = [&](int E, int64_t L) -> int64_t {
    const auto &b = bucket[E];
    return std::partition_point(b.begin(), b.end(), [&](int32_t j) { return Ly[j] >= L; }) - b.begin();
  };

  // Chosen form: libraries up to kGramLMax samples use the filter for E >= kGramEMin.
  const bool chosen = ctx->form == EDM_FORM_CHOSEN;
  auto filt_of = [&](int64_t i) { return chosen && Lx[i] <= edm::kGramLMax; };

  // Libraries longest first; per library the E it needs and their table sizes.
  std::vector<int32_t> order(static_cast<size_t>(Nl));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t u, int32_t v) { return Lx[u] > Lx[v]; });
  std::vector<uint32_t> need(static_cast<size_t>(Nl), 0);
  std::vector<int64_t> bytes(static_cast<size_t>(Nl), 0);
  for (int64_t i = 0; i < Nl; ++i) {
    for (int E = 1; E <= EDM_E_MAX; ++E) {
      const int64_t m = Lx[i] - (E - 1) - Tp;
      if (m - 1 >= E + 1 && defined(E, Lx[i]) > 0) {
        need[static_cast<size_t>(i)] |= 1u << (E - 1);
        bytes[static_cast<size_t>(i)] += static_cast<int64_t>(align_up(static_cast<size_t>(m) * (E + 1) * 4, 256));
      }
    }
  }
  // Batches: consecutive libraries (in that order) whose tables fit the limit.
  const int64_t limit = static_cast<int64_t>(workspace_limit());
  std::vector<int64_t> tbl_off(static_cast<size_t>(Nl) * (EDM_E_MAX + 1), 0);
  std::vector<edm::TableItem> titems;
  std::vector<edm::LookupItem> litems;
  std::vector<int32_t> item_libs;
  int64_t max_batch_elems = 0;
  int64_t k = 0;
  while (k < Nl) {
    Batch B;
    int64_t elems = 0;
    const int64_t k0 = k;
    while (k < Nl) {
      const int32_t i = order[static_cast<size_t>(k)];
      const int64_t e = bytes[static_cast<size_t>(i)] / 4;
      if (k > k0 && (elems + e) * 8 > limit) break;
      elems += e;
      ++k;
    }
    if (elems * 8 > limit) {
      edm_ccm_plan_destroy(nullptr, P);
      return set_err(ctx, EDM_E_NOMEM, "one library's tables exceed EDM_WORKSPACE_LIMIT");
    }
    max_batch_elems = std::max(max_batch_elems, elems);
    // table offsets (elements) inside the batch's table buffer
    int64_t o = 0;
    for (int64_t q = k0; q < k; ++q) {
      const int32_t i = order[static_cast<size_t>(q)];
      B.L_max = std::max(B.L_max, Lx[i]);
      if (filt_of(i)) B.Lg_max = std::max(B.Lg_max, Lx[i]);
      if (filt_of(i) && Lx[i] <= edm::kGramLdsXsMax) B.Ls_max = std::max(B.Ls_max, Lx[i]);
      for (int E = 1; E <= EDM_E_MAX; ++E) {
        if (!((need[static_cast<size_t>(i)] >> (E - 1)) & 1u)) continue;
        tbl_off[static_cast<size_t>(i) * (EDM_E_MAX + 1) + E] = o;
        const int64_t m = Lx[i] - (E - 1) - Tp;
        o += static_cast<int64_t>(align_up(static_cast<size_t>(m) * (E + 1) * 4, 256)) / 4;
      }
    }
    // table items, per list, longest library first (a filtered block also
    // covers kKnnThreads queries)
    for (int c = 0; c < kNLists; ++c) {
      B.t_begin[c] = static_cast<int64_t>(titems.size());
      for (int64_t q = k0; q < k; ++q) {
        const int32_t i = order[static_cast<size_t>(q)];
        int lo = 0, hi = 0;
        if (!list_range(c, filt_of(i), Lx[i] > edm::kGramLdsXsMax, lo, hi)) continue;
        uint32_t gm = 0;
        for (int E = lo; E <= hi; ++E) gm |= need[static_cast<size_t>(i)] & (1u << (E - 1));
        if (!gm) continue;
        const int64_t m_lo = Lx[i] - (lo - 1) - Tp;
        const int64_t nb = (m_lo + edm::kKnnThreads - 1) / edm::kKnnThreads;
        for (int64_t b = 0; b < nb; ++b)
          titems.push_back(edm::TableItem{i, static_cast<int16_t>(c), static_cast<int16_t>(b)});
      }
      B.t_count[c] = static_cast<int64_t>(titems.size()) - B.t_begin[c];
    }
    // lookup items, per E: groups of consecutive libraries (longest first)
    // that need E, each against tiles of the targets its shortest library
    // pairs with (a prefix of the bucket; a longer library skips the targets
    // shorter than itself)
    for (int E = 1; E <= EDM_E_MAX; ++E) {
      B.l_begin[E] = static_cast<int64_t>(litems.size());
      std::vector<int32_t> grp;
      auto close_group = [&]() {
        if (grp.empty()) return;
        const int64_t m = Lx[grp.front()] - (E - 1) - Tp;  // the longest window
        const int64_t cnt = defined(E, Lx[grp.back()]);
        // staged targets of an item: a power of two up to the tune's count
        // whose tile fits the lookup kernel's LDS
        int64_t T = edm::lookup_tile_targets(m);
        while (T > tn.lookup_targets) T >>= 1;
        B.lds_floats[E] = std::max(B.lds_floats[E], edm::lookup_tile_floats(static_cast<int>(T), m));
        const int32_t at = static_cast<int32_t>(item_libs.size());
        item_libs.insert(item_libs.end(), grp.begin(), grp.end());
        for (int64_t f = 0; f < cnt; f += T)
          litems.push_back(edm::LookupItem{at, static_cast<int16_t>(grp.size()), static_cast<int16_t>(T),
                                           static_cast<int32_t>(f), static_cast<int32_t>(std::min(T, cnt - f))});
        grp.clear();
      };
      for (int64_t q = k0; q < k; ++q) {
        const int32_t i = order[static_cast<size_t>(q)];
        if (!((need[static_cast<size_t>(i)] >> (E - 1)) & 1u)) continue;
        grp.push_back(i);
        if (static_cast<int>(grp.size()) == edm::kLookupItemLibs) close_group();
      }
      close_group();
      B.l_count[E] = static_cast<int64_t>(litems.size()) - B.l_begin[E];
    }
    P->batches.push_back(B);
  }
  P->n_counters = static_cast<int>(P->batches.size()) * (kNLists + EDM_E_MAX);
  for (const Batch &B : P->batches) P->Lg_max = std::max(P->Lg_max, B.Lg_max);
  P->filtered = P->Lg_max > 0;
  P->gram_ld = P->filtered ? edm::gram_ld(P->Lg_max) : 0;

  // One device allocation: lengths, masks, offsets, buckets, counters,
  // items, and the table buffer of the largest batch.
  Plan lay;
  const size_t oLx = lay.take(sizeof(int64_t) * Nl);
  const size_t oLy = lay.take(sizeof(int64_t) * Nt);
  const size_t oNeed = lay.take(sizeof(uint32_t) * Nl);
  const size_t oOff = lay.take(sizeof(int64_t) * tbl_off.size());
  const size_t oIds = lay.take(sizeof(int32_t) * std::max<size_t>(ids.size(), 1));
  const size_t oAt = lay.take(sizeof(int32_t) * at.size());
  const size_t oCnt = lay.take(sizeof(int) * P->n_counters);
  const size_t oTi = lay.take(sizeof(edm::TableItem) * std::max<size_t>(titems.size(), 1));
  const size_t oLi = lay.take(sizeof(edm::LookupItem) * std::max<size_t>(litems.size(), 1));
  const size_t oIl = lay.take(sizeof(int32_t) * std::max<size_t>(item_libs.size(), 1));
  const size_t small = lay.bytes;
  const size_t oTidx = lay.take(sizeof(int32_t) * max_batch_elems);
  const size_t oTw = lay.take(sizeof(float) * max_batch_elems);
  // filter prep of every library: centring constants and packed norms
  const size_t oCm = lay.take(sizeof(float) * Nt);
  const size_t oGmu = P->filtered ? lay.take(sizeof(float) * Nl) : 0;
  const size_t oGnrm =
      P->filtered ? lay.take(sizeof(uint32_t) * static_cast<size_t>(Nl) * edm::kGramNE * P->gram_ld) : 0;
  if (hipMalloc(reinterpret_cast<void **>(&P->dev), lay.bytes) != hipSuccess) {
    (void)hipGetLastError();
    P->dev = nullptr;
    edm_ccm_plan_destroy(nullptr, P);
    return set_err(ctx, EDM_E_NOMEM, "plan allocation of " + std::to_string(lay.bytes) + " bytes failed");
  }
  P->Lx_dev = reinterpret_cast<int64_t *>(P->dev + oLx);
  P->Ly_dev = reinterpret_cast<int64_t *>(P->dev + oLy);
  P->need = reinterpret_cast<uint32_t *>(P->dev + oNeed);
  P->tbl_off = reinterpret_cast<int64_t *>(P->dev + oOff);
  P->bucket_ids = reinterpret_cast<int32_t *>(P->dev + oIds);
  P->bucket_at = reinterpret_cast<int32_t *>(P->dev + oAt);
  P->counters = reinterpret_cast<int *>(P->dev + oCnt);
  P->titems = reinterpret_cast<edm::TableItem *>(P->dev + oTi);
  P->litems = reinterpret_cast<edm::LookupItem *>(P->dev + oLi);
  P->item_libs = reinterpret_cast<int32_t *>(P->dev + oIl);
  P->tbl_idx = reinterpret_cast<int32_t *>(P->dev + oTidx);
  P->tbl_w = reinterpret_cast<float *>(P->dev + oTw);
  P->cmean = reinterpret_cast<float *>(P->dev + oCm);
  if (P->filtered) {
    P->gram_mu = reinterpret_cast<float *>(P->dev + oGmu);
    P->gram_nrm = reinterpret_cast<uint32_t *>(P->dev + oGnrm);
  }
  std::vector<char> blob(small, 0);
  std::memcpy(blob.data() + oLx, Lx, sizeof(int64_t) * Nl);
  std::memcpy(blob.data() + oLy, Ly, sizeof(int64_t) * Nt);
  std::memcpy(blob.data() + oNeed, need.data(), sizeof(uint32_t) * Nl);
  std::memcpy(blob.data() + oOff, tbl_off.data(), sizeof(int64_t) * tbl_off.size());
  if (!ids.empty()) std::memcpy(blob.data() + oIds, ids.data(), sizeof(int32_t) * ids.size());
  std::memcpy(blob.data() + oAt, at.data(), sizeof(int32_t) * at.size());
  if (!titems.empty()) std::memcpy(blob.data() + oTi, titems.data(), sizeof(edm::TableItem) * titems.size());
  if (!litems.empty()) std::memcpy(blob.data() + oLi, litems.data(), sizeof(edm::LookupItem) * litems.size());
  if (!item_libs.empty()) std::memcpy(blob.data() + oIl, item_libs.data(), sizeof(int32_t) * item_libs.size());
  int rc = upload(ctx, blob.data(), small, P->dev);
  if (rc == EDM_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = set_err(ctx, EDM_E_HIP, "plan upload failed");
  if (rc != EDM_OK) {
    edm_ccm_plan_destroy(nullptr, P);
    return rc;
  }
  *out = P;
  return EDM_OK;
}

}  // extern "C"

namespace {

// Enqueue one run of the plan on the stream (what the graph captures).
int enqueue_plan(edm_ctx *ctx, edm_plan *P, const float *X, const float *Y, float *rho) {
  const hipStream_t st = ctx->stream;
  EDM_HIP(ctx, edm::launch_fill(rho, P->Nl * P->Nt, __builtin_nanf(""), st));
  // counters start at 0: an all-zero float fill writes zero bits
  EDM_HIP(ctx, edm::launch_fill(reinterpret_cast<float *>(P->counters), P->n_counters, 0.0f, st));
  EDM_HIP(ctx, edm::launch_target_means(Y, P->ldy, P->Ly_dev, 0, P->Nt, P->cmean, st));
  edm::KnnArgs a{};
  a.X = X;
  a.ldx = P->ldx;
  a.L_dev = P->Lx_dev;
  a.tau = 1;
  a.Tp = P->Tp;
  a.E_max = EDM_E_MAX;
  a.status = ctx->status;
  a.need_dev = P->need;
  a.tbl_off = P->tbl_off;
  a.tbl_idx = P->tbl_idx;
  a.tbl_w = P->tbl_w;
  if (P->filtered) {
    a.gram_mu = P->gram_mu;
    a.gram_nrm = P->gram_nrm;
    a.gram_ld = P->gram_ld;
    EDM_HIP(ctx, edm::launch_gram_prep(a, static_cast<int>(P->Nl), P->Lg_max, st));
  }
  int c = 0;
  for (const Batch &B : P->batches) {
    for (int g = 0; g <= kNGroups; ++g, ++c)
      EDM_HIP(ctx, edm::launch_tables_persistent(a, g, P->titems + B.t_begin[g], static_cast<int>(B.t_count[g]),
                                                 P->counters + c, B.L_max, P->tune.tables_wg_per_cu,
                                                 P->n_cu, st));
    for (int h = 0; h < 2; ++h) {  // short libraries (LDS stride of the short ones), then long ones
      edm::KnnArgs ah = a;
      ah.p1_stride = P->tune.filter_stride;
      const int64_t Lh = h == 0 ? B.Ls_max : B.Lg_max;
      ah.gram_lds = Lh > 0 ? edm::gram_ld(Lh) : 0;
      for (int f = 0; f < kNGram; ++f, ++c) {
        const int l = kNGroups + 1 + h * kNGram + f;
        EDM_HIP(ctx, edm::launch_gram_items(ah, f, P->titems + B.t_begin[l], static_cast<int>(B.t_count[l]),
                                            Lh, st));
      }
    }
    edm::LookupArgs b{};
    b.Lx_dev = P->Lx_dev;
    b.tau = 1;
    b.Tp = P->Tp;
    b.Y = Y;
    b.cmean = P->cmean;
    b.ldy = P->ldy;
    b.Ly_dev = P->Ly_dev;
    b.rho = rho;
    b.ldrho = P->Nt;
    b.status = ctx->status;
    b.tbl_off = P->tbl_off;
    b.tbl_idx = P->tbl_idx;
    b.tbl_w = P->tbl_w;
    b.bucket_ids = P->bucket_ids;
    b.bucket_at = P->bucket_at;
    b.item_libs = P->item_libs;
    for (int E = 1; E <= EDM_E_MAX; ++E, ++c)
      EDM_HIP(ctx, edm::launch_lookup_items(b, E, P->litems + B.l_begin[E], static_cast<int>(B.l_count[E]),
                                            P->counters + c, B.lds_floats[E], P->tune.lookup_wg_per_cu,
                                            P->n_cu, st));
  }
  return EDM_OK;
}

}  // namespace

extern "C" int edm_ccm_plan_run(edm_ctx *ctx, edm_plan *P, const float *X, const float *Y,
                                float *rho) {
  if (!P || !X || !Y || !rho) return set_err(ctx, EDM_E_ARG, "NULL pointer");
  EDM_RC(check_ctx(ctx));
  if (ctx->stream == nullptr) return enqueue_plan(ctx, P, X, Y, rho);  // no capture on the legacy stream
  if (!P->exec || P->gX != X || P->gY != Y || P->grho != rho || P->gstream != ctx->stream) {
    if (P->exec) {
      (void)hipGraphExecDestroy(P->exec);
      P->exec = nullptr;
    }
    if (P->graph) {
      (void)hipGraphDestroy(P->graph);
      P->graph = nullptr;
    }
    EDM_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
    const int rc = enqueue_plan(ctx, P, X, Y, rho);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (rc != EDM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamEndCapture");
    P->graph = g;
    EDM_HIP(ctx, hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    P->gX = X;
    P->gY = Y;
    P->grho = rho;
    P->gstream = ctx->stream;
  }
  TimingScope timing_scope(ctx);
  edm::TimedLaunch timed(EDM_KF_PLAN, ctx->stream);
  EDM_HIP(ctx, hipGraphLaunch(P->exec, ctx->stream));
  return EDM_OK;
}
