// Internal interface between the host orchestration (edm_api.hip) and the
// kernel files.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/edm.h"

namespace edm {

struct Mom;

// Records a HIP event pair on `st` around the launches made during its
// lifetime and attributes them to kernel family `family` (EDM_KF_*), when
// the calling thread is inside a TimingScope of a context with timing on;
// otherwise does nothing.
struct TimedLaunch {
  TimedLaunch(int family, hipStream_t st);
  ~TimedLaunch();
  int family;
  hipStream_t st;
  hipEvent_t start = nullptr;
};

constexpr int kKnnThreads = 256;  // 4 waves of 64 query points per workgroup

// Arguments of the fused embedding + distance + top-k + weights kernel.
// One workgroup handles 256 consecutive query points of one library; the
// grid's y index is the library slot.
struct KnnArgs {
  const float *X;            // libraries, row `row` at X + row*ldx
  int64_t ldx;
  const int64_t *L_dev;      // per-row lengths (device) or nullptr -> L_uni
  int64_t L_uni;
  const int32_t *lib_ids;    // slot -> row of X (device) or nullptr -> row = slot
  int32_t E, tau, Tp, k;
  int32_t excl;              // exclusion radius: candidates with |q - p| <= excl are skipped
  int32_t p1_stride;         // filter pass 1 visits one candidate tile in p1_stride (0: by group and length)
  int32_t *idx;              // [slot][nq][k] or nullptr
  float *dist;               // [slot][nq][k] or nullptr
  float *w;                  // [slot][nq][k] or nullptr
  int64_t tbl_stride;        // elements between consecutive slots' tables
  Mom *mom;                  // sweep: per-block co-moments of the self-prediction, or nullptr
  int32_t mom_blocks;        // blocks per (row, E) in mom
  int32_t E_max;             // sweep: number of E slots per row in mom
  int *status;               // device status word (bit 0: non-finite input)
  // Batched kernel, table mode: bit E-1 of need marks the E whose tables are
  // written to idxE[E] / wE[E] ([slot][nq][E+1], slot stride strideE[E]).
  uint32_t need;
  int32_t *idxE[EDM_E_MAX + 1];
  float *wE[EDM_E_MAX + 1];
  int64_t strideE[EDM_E_MAX + 1];
  // Plan mode (persistent kernel): per-row need masks and table offsets
  // (elements, [row][EDM_E_MAX + 1]) into tbl_idx / tbl_w.
  const uint32_t *need_dev;
  const int64_t *tbl_off;
  int32_t *tbl_idx;
  float *tbl_w;
  // Matrix-core filter (chosen form, E >= kGramEMin): per-slot centring
  // constants and packed BF16 hi/lo norms, [slot][E - kGramEMin][gram_ld]
  // (written by launch_gram_prep).  gram_nrm == nullptr selects the exact
  // scan for every E.
  float *gram_mu;
  uint32_t *gram_nrm;
  int64_t gram_ld;
  int64_t gram_lds;  // LDS row stride of a launch (0: gram_ld); >= its rows' L + kGramPad
  // Sweep mode: when keepE[E] is set, the sorted neighbour list of every
  // query at E is also written there ([slot][m][E+1] int32, slot stride
  // keep_strideE[E]) for a later cross map (launch_tables_from_sweep).
  // keepWE[E] (same layout, float32, or nullptr): the list's normalised
  // weights, which are the cross map's weights wherever its list is the same.
  int32_t *keepE[EDM_E_MAX + 1];
  float *keepWE[EDM_E_MAX + 1];
  int64_t keep_strideE[EDM_E_MAX + 1];
  // Cross map with the targets grouped on the device (launch_group_by_E):
  // bucket offsets [EDM_E_MAX + 2]; a table kernel of dimension E exits when
  // bucket E is empty.  nullptr: every launched table is built.
  const int32_t *group_at;
};

// Work item of the persistent table kernel: E group and query block of a row.
struct TableItem {
  int32_t row;
  int16_t group;
  int16_t blk;
};

// Work item of the lookup work-list kernel: a tile of targets of one E
// (bucket_ids[bucket_at[E] + first ...]) against a group of up to
// kLookupItemLibs libraries (LookupArgs::item_libs[lib ... lib + nlib - 1],
// longest first), one wave per library.
constexpr int kLookupItemMaxTargets = 16;  // T of a LookupItem: 1, 2, 4, 8 or 16
constexpr int kLookupItemLibs = 16;        // libraries of a LookupItem, at most
struct LookupItem {
  int32_t lib;    // first entry of the item's libraries in item_libs
  int16_t nlib;   // libraries of the item (1 .. kLookupItemLibs)
  int16_t T;      // targets staged per tile
  int32_t first;  // index of the tile's first target inside the E bucket
  int32_t count;  // targets in this tile
};

// Persistent table kernel of one E group (0: E 1-8, 1: 9-12, 2: 13-15,
// 3: 16-18, 4: 19-20) over its work list (counter: a device int that starts
// at 0).
// group: 0-4 the exact E groups {1-8, 9-12, 13-15, 16-18, 19-20}; 5: E 1-4.
hipError_t launch_tables_persistent(const KnnArgs &a, int group, const TableItem *items,
                                    int n_items, int *counter, int64_t L_max, int wg_per_cu,
                                    int n_cu, hipStream_t st);

// Matrix-core filter of the batched scans (gram.hip).  E values from
// kGramEMin up run through it when KnnArgs::gram_nrm is set; kGramLMax bounds
// the series length (LDS holds the BF16 halves of the series, and its float32
// samples up to kGramLdsXsMax).
constexpr int kGramEMin = 5;
constexpr int kGramNE = EDM_E_MAX - kGramEMin + 1;
constexpr int kGramPad = 64;  // zero samples staged past the end of a series
constexpr int64_t kGramLMax = 32000;      // longest series of the filtered scan (LDS budget)
constexpr int64_t kGramLdsXsMax = 14336;  // longer: exact samples read from global memory
// E groups of the filtered scan (one register list per E of a group; the
// slot layout needs E_hi + |group| + 1 <= 16 or a shared first chunk).
constexpr int kGramGroups[6][2] = {{5, 8}, {9, 11}, {12, 13}, {14, 16}, {17, 18}, {19, 20}};
inline int64_t gram_ld(int64_t L_max) { return (L_max + kGramPad + 63) / 64 * 64; }
// Per slot: centring constant, then the packed norms of every E >= kGramEMin.
hipError_t launch_gram_prep(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st);
// Batched scan of one E range [lo, hi] (lo >= kGramEMin) through the filter;
// same outputs as launch_sweep_multi.
hipError_t launch_gram_group(const KnnArgs &a, int lo, int hi, int nslots, int64_t L_max,
                             hipStream_t st);
// Work-list form for the plan: items (row, blk) of filtered group g
// (kGramGroups[g]), table mode, one workgroup per item; same outputs as
// launch_tables_persistent.  L_max bounds the rows of the items; a.gram_ld
// and the LDS stride a.gram_lds (0: gram_ld) must be >= L_max + kGramPad.
hipError_t launch_gram_items(const KnnArgs &a, int g, const TableItem *items, int n_items,
                             int64_t L_max, hipStream_t st);

// Cross-map tables (Tp = 0) of dimension E for `nslots` libraries from the
// sweep's lists (Tp = 1) in a.keepE[E]; output in a.idxE[E] / a.wE[E] with
// a.strideE[E], as the batched table mode writes them.
hipError_t launch_tables_from_sweep(const KnnArgs &a, int E, int nslots, int64_t L_max,
                                    hipStream_t st);

// Launch the kNN kernel for `nslots` libraries whose longest series has
// `L_max` samples.  Returns a hipError_t.
hipError_t launch_knn(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st);

// Tables of one library (a.X, a.L_uni, tau, Tp, E, k = E+1, a.excl) whose
// candidates are restricted to subsamples: set s holds the ascending member
// indices sets[off[s] .. off[s+1]) (device), table s goes to a.idx / a.w +
// s * a.tbl_stride ([m][k]).
hipError_t launch_knn_subsets(const KnnArgs &a, const int32_t *sets, const int64_t *off, int n_sets,
                              hipStream_t st);

// The paper's two-kernel form of launch_knn (same outputs): per pass of up to
// slots_per_pass libraries, the distance matrices [slot][m][ldd] float32 are
// written to D (Algorithm 1), then each row's k smallest are selected
// (Algorithm 2) and finished as the fused kernel does.  D must hold
// slots_per_pass * ldd * ldd floats; ldd = two_kernel_ld(m_max) with
// m_max = L_max - (E-1)*tau - Tp.
int64_t two_kernel_ld(int64_t m_max);
hipError_t launch_knn_two_kernel(const KnnArgs &a, int nslots, int64_t L_max, float *D, int64_t ldd,
                                 int slots_per_pass, hipStream_t st);

// Batched kNN (tau = 1): one scan per group of E values.  With a.mom set it
// writes the sweep's per-block co-moments for E = 1..a.E_max; otherwise it
// writes the tables of every E marked in a.need.  Outputs are bit-identical to
// launch_knn per E.
hipError_t launch_sweep_multi(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st);

// Arguments of the batched lookup + on-the-fly Pearson kernel.  One
// workgroup handles one library table and a tile of targets.
struct LookupArgs {
  const int32_t *idx;        // [slot][nq][k]
  const float *w;            // [slot][nq][k]
  int64_t tbl_stride;
  const int32_t *lib_ids;    // slot -> library id (rho row, Lx index); nullptr -> slot
  const int64_t *Lx_dev;     // library lengths (device) or nullptr -> Lx_uni
  int64_t Lx_uni;
  int32_t E, tau, Tp, k;
  int32_t excl;              // exclusion radius of the tables (a table exists iff m-1-2*excl >= k)
  const float *Y;            // targets, row j at Y + j*ldy
  const float *cmean;        // centring constant of every target (launch_target_means)
  int64_t ldy;
  const int64_t *Ly_dev;     // target lengths (device) or nullptr -> every target long enough
  const int32_t *tgt_ids;    // bucket position -> target id (device) or nullptr -> identity
  int32_t ntgt;
  float *rho;                // rho[lib*ldrho + tgt] or nullptr
  int64_t ldrho;
  float *pred;               // pred[tgt*ldpred + p] (single table only) or nullptr
  int64_t ldpred;
  int *status;
  // Plan mode (item kernels): tables at tbl_off[lib][E] in tbl_idx / tbl_w,
  // targets of E listed at bucket_ids[bucket_at[E] ...].
  const int64_t *tbl_off;
  const int32_t *tbl_idx;
  const float *tbl_w;
  const int32_t *bucket_ids;
  const int32_t *bucket_at;
  const int32_t *item_libs;  // library ids of the work items' groups
  // Grid kernel with the bucket on the device (tbl_off == nullptr and
  // bucket_at set): the targets are bucket_ids[bucket_at[E] ..
  // bucket_at[E+1]) and ntgt is ignored.
};

// Lookups of the work list of one E: persistent (wg_per_cu * n_cu
// workgroups pulling items from *counter) or one workgroup per item
// (wg_per_cu = 0).
// lds_floats: dynamic LDS per workgroup (max over items of lookup_tile_floats).
hipError_t launch_lookup_items(const LookupArgs &a, int E, const LookupItem *items, int n_items,
                               int *counter, int64_t lds_floats, int wg_per_cu, int n_cu,
                               hipStream_t st);

hipError_t launch_lookup(const LookupArgs &a, int nslots, int64_t m_max, hipStream_t st);

// Centring constants of targets Y[N][ldy] for the lookups: the float32 of each
// target's float64 mean over [0, Ly_dev[t]) (or [0, L_uni)).
hipError_t launch_target_means(const float *Y, int64_t ldy, const int64_t *Ly_dev, int64_t L_uni,
                               int64_t N, float *cmean, hipStream_t st);

// Targets per staged lookup tile for a window of m samples: the largest of
// 16, 8, 4, 2, 1 whose tile fits the lookup kernels' 160 KB of LDS.
int lookup_tile_targets(int64_t m);
// LDS floats of a staged tile of T targets over a window of m samples
// (padded rows).
int64_t lookup_tile_floats(int T, int64_t m);

// Sweep epilogue: merge the per-block moments into rho[N][E_max] and pick
// E_opt (smallest E with the largest non-NaN rho).
// cand: optional per-series bit set of the E values evaluated (nullptr: all).
hipError_t launch_sweep_finalize(const Mom *mom, int32_t mom_blocks, const int64_t *L_dev,
                                 int64_t N, int32_t E_max, int32_t tau, int32_t Tp, int32_t excl,
                                 const uint32_t *cand, float *rho, int32_t *E_opt,
                                 hipStream_t st);
hipError_t launch_candidates(const float *logits, int64_t N, int32_t E_max, int32_t m_top,
                             float min_conf, uint32_t *cand, hipStream_t st);

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t st);
// Stable grouping of N targets by E (counting sort on the device): at[e] is
// the first position of bucket e (e = 0 holds E outside 1..E_max), at[E_max+1
// .. EDM_E_MAX+1] = N, ids[at[e] ..] the targets of E in ascending order.
hipError_t launch_group_by_E(const int32_t *E, int64_t N, int32_t E_max, int32_t *at, int32_t *ids,
                             hipStream_t st);
// launch_lookup with the bucket on the device: a.bucket_ids / a.bucket_at
// set, n_tgt_max bounds the bucket (for the tile size).
hipError_t launch_lookup_bucket(const LookupArgs &a, int nslots, int64_t m_max, int64_t n_tgt_max,
                                hipStream_t st);
// Rows of `words` 32-bit words: gather dst[i] = src[ids[i]] or scatter
// dst[ids[i]] = src[i], i < n; leading dimensions in words.
hipError_t launch_copy_rows(const void *src, int64_t lds, void *dst, int64_t ldd, const int32_t *ids,
                            int64_t n, int64_t words, bool scatter, hipStream_t st);
hipError_t launch_embed(const float *x, int64_t L, int32_t E, int32_t tau, float *out,
                        int *status, hipStream_t st);

// Size in bytes of one Mom record (for workspace sizing on the host).
constexpr size_t kMomBytes = 6 * sizeof(double);

}  // namespace edm
