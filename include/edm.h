/*
 * edm.h -- C ABI of libedm, all-to-all convergent cross mapping (CCM) on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those of the kEDM paper (Takahashi et al., PEARC '21):
 * Section 2.1 steps 1-4 (embedding, k-nearest-neighbour search, simplex
 * lookup, Pearson skill), Section 3.3 Algorithms 1-2 (all-kNN table:
 * pairwise distances, then the k smallest of each row, normalised) and
 * Section 3.4 Algorithm 3 (batched lookup of every target through a
 * library's table, targets grouped by their optimal embedding dimension,
 * correlation computed without writing predictions).
 *
 * Conventions for every call
 * --------------------------
 * - Array pointers are DEVICE pointers (hipMalloc / torch CUDA tensors)
 *   unless marked (host).  Arrays are row-major and C-contiguous in their
 *   last dimension.  The caller owns every buffer it passes; libedm owns
 *   only the workspace inside an edm_ctx.
 * - Every call returns EDM_OK or a negative EDM_E_* code.  Arguments are
 *   validated on the host before anything is enqueued, so an error return
 *   means nothing was written.  No C++ exception crosses the ABI.
 * - Work is enqueued asynchronously on the context's stream; outputs are
 *   valid after edm_sync() or a synchronisation of that stream.  Exception:
 *   edm_simplex_sweep and edm_ccm copy small host arrays to the device and
 *   edm_ccm reads E_tgt back to the host (one stream synchronisation).
 * - One context per stream.  Calls on one context must not overlap in time
 *   from several host threads.
 * - Inputs must be finite.  Kernels that read a series flag any non-finite
 *   sample in a device status word, and edm_sync() then returns
 *   EDM_E_NONFINITE (outputs for such series are unspecified).
 *
 * Notation
 * --------
 * A series x of length L, embedding dimension E >= 1, lag tau >= 1, horizon
 * Tp >= 0.  Embedded point p has coordinates v_p[j] = x[p + j*tau],
 * j = 0..E-1, and time stamp t(p) = p + (E-1)*tau; there are
 * n = L - (E-1)*tau of them.  Query points and candidate neighbours are both
 * p in [0, nq) with nq = n - Tp, so that a neighbour's future value exists.
 * The neighbour ranking key is the float32 squared distance of Algorithm 1,
 * sum over j ascending of (x[p+j*tau] - x[q+j*tau])^2 with one float32
 * rounding after every subtraction, product and sum; ties are broken by the
 * lower index q; q = p is excluded.  A call needs nq - 1 >= k, otherwise it
 * returns EDM_E_SHORT.
 */
#ifndef EDM_H
#define EDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct edm_ctx edm_ctx;

/* Form of the computation (results are identical; only the schedule differs).
 * EDM_FORM_PLAIN  : one candidate scan per (library, E), float32 VALU keys.
 * EDM_FORM_BATCHED: with tau = 1, edm_simplex_sweep and edm_ccm run one
 *                   candidate scan per group of E values, extending one
 *                   running key (the key for E is the key for E-1 plus one
 *                   rounded term).
 * EDM_FORM_CHOSEN : EDM_FORM_BATCHED, and for E >= 5 (series up to 32000
 *                   samples) a BF16 matrix-core estimate of every key filters
 *                   the candidates; the ones that may enter a top-k list are
 *                   re-ranked with the exact float32 key.
 * EDM_FORM_TWO_KERNEL: the paper's own form of the kNN step (Section 3.3):
 *                   Algorithm 1 writes each library's whole distance matrix
 *                   (float32 keys, m x m) to device memory, then Algorithm 2
 *                   selects the k smallest of every row.  Used by edm_knn,
 *                   edm_simplex_sweep, edm_ccm, edm_sweep_ccm and
 *                   edm_select_E in place of the fused scan; the matrices of
 *                   up to 2 GiB of libraries at a time (at least one) live
 *                   in a context buffer (EDM_E_NOMEM beyond the workspace
 *                   limit).  Batched plans treat it as EDM_FORM_PLAIN.
 * Tables, rho and E_opt are bit-identical across the forms. */
typedef enum {
  EDM_FORM_PLAIN = 0,
  EDM_FORM_CHOSEN = 1,
  EDM_FORM_BATCHED = 2,
  EDM_FORM_TWO_KERNEL = 3
} edm_form;

enum {
  EDM_OK = 0,
  EDM_E_ARG = -1,       /* invalid argument (NULL pointer, E/tau/Tp/k/ld out of range) */
  EDM_E_SHORT = -2,     /* series too short: nq - 1 < k                              */
  EDM_E_HIP = -3,       /* a HIP runtime call or kernel failed                       */
  EDM_E_NOMEM = -4,     /* workspace allocation failed                               */
  EDM_E_NONFINITE = -5  /* a kernel saw a non-finite input sample (from edm_sync)    */
};

/* Largest supported embedding dimension of the fast path and for the sweep. */
#define EDM_E_MAX 20
/* Largest supported neighbour count k. */
#define EDM_K_MAX 32
/* Longest supported series (samples); a library series is staged whole in
 * the 160 KiB local data share of one compute unit. */
#define EDM_L_MAX 32768

/* Create a context bound to an existing HIP stream (a hipStream_t passed as
 * void*; NULL means the default stream).  The stream is borrowed, never
 * destroyed by libedm.  The current HIP device at creation is the context's
 * device.  Returns EDM_E_HIP when no device is usable. */
int edm_ctx_create(edm_ctx **ctx, void *hip_stream);

/* Select the arithmetic form (edm_form) for later calls. */
int edm_ctx_set_form(edm_ctx *ctx, int form);

/* Exclusion radius r >= 0 of the neighbour search for later calls on ctx
 * (default 0): candidates q with |q - p| <= r are never neighbours of query
 * p (r = 0 excludes only q = p, the method of Section 2.1 step 2; a larger
 * r is a Theiler window, which the paper does not use).  A table needs
 * nq - 1 - 2r >= k (edm_knn returns EDM_E_SHORT otherwise; in sweeps and
 * cross maps such an E or pair is NaN).  With r > 0, edm_simplex_sweep,
 * edm_ccm and edm_sweep_ccm run the per-E scan of EDM_FORM_PLAIN (or the
 * two-kernel form) whatever the form, and edm_ccm_plan_create returns
 * EDM_E_ARG.  Returns EDM_E_ARG for r < 0 or r > EDM_L_MAX. */
int edm_ctx_set_exclusion_radius(edm_ctx *ctx, int32_t r);

/* Wait for the context's stream.  Returns EDM_E_HIP for an asynchronous
 * kernel error and EDM_E_NONFINITE when a kernel flagged a non-finite input
 * since the previous edm_sync (the flag is then cleared). */
int edm_sync(edm_ctx *ctx);

/* Text of the last error on ctx (never NULL; valid until the next call on
 * ctx).  With ctx == NULL, the last error of edm_ctx_create on this thread. */
const char *edm_last_error(const edm_ctx *ctx);

/* Release the workspace and the context.  Synchronises its stream first. */
void edm_ctx_destroy(edm_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Kernel timing.  With timing on, every call on the context records a pair
 * of HIP events on its stream around each kernel launch and attributes the
 * time to one kernel family.  Launches inside a captured plan graph are not
 * timed.  Timing adds two event records per launch; it is off by default.
 * ------------------------------------------------------------------------- */
enum {
  EDM_KF_EXACT_SCAN = 0,        /* k_knn: one candidate scan per (library, E)        */
  EDM_KF_BATCHED_SCAN = 1,      /* k_sweep_multi, k_tables_persistent: exact scans
                                   of groups of E values                            */
  EDM_KF_FILTER_PREP = 2,       /* k_gram_mean, k_gram_norms                         */
  EDM_KF_FILTER_SCAN = 3,       /* k_gram, k_gram_items: matrix-core filtered scans  */
  EDM_KF_TABLES_FROM_SWEEP = 4, /* k_fix_from_sweep, k_scan_queries                  */
  EDM_KF_LOOKUP = 5,            /* k_lookup, k_lookup_items                          */
  EDM_KF_FINALIZE = 6,          /* k_sweep_finalize                                  */
  EDM_KF_OTHER = 7,             /* fills, embedding, candidate sets, network         */
  EDM_KF_DISTANCES = 8,         /* two-kernel form: distance matrix (Algorithm 1)    */
  EDM_KF_ROW_TOPK = 9,          /* two-kernel form: per-row top-k (Algorithm 2)      */
  EDM_KF_GROUP = 10,            /* grouping of targets by E on the device            */
  EDM_KF_PLAN = 11,             /* one replay of a batched plan's graph, as a whole  */
  EDM_KF_COUNT = 12
};

/* Switch timing on (on != 0) or off; either way the accumulated times are
 * cleared. */
int edm_ctx_set_timing(edm_ctx *ctx, int on);

/* Wait for the context's stream, then add the time (milliseconds) and the
 * number of launches recorded per family since the last call (or since
 * edm_ctx_set_timing) into ms[EDM_KF_COUNT] and launches[EDM_KF_COUNT]
 * (host arrays; either may be NULL) and clear the records. */
int edm_ctx_timing(edm_ctx *ctx, double *ms, int64_t *launches);

/* Empirical ceilings of the device, measured with the library's own kernels
 * on the context's stream (Section 4.4 builds its rooflines from measured
 * ceilings): HBM streaming bandwidth of a vectorised copy of 2 GiB (bytes
 * read + written per second, GB/s), BF16 matrix-core throughput of
 * independent v_mfma_f32_32x32x16_bf16 chains (TFLOP/s, 2 flops per
 * multiply-add) and float32 vector throughput of independent non-fused
 * additions (T ops/s).  Uses 4 GiB of workspace; synchronises the stream.
 * Outputs are host doubles. */
int edm_ceilings(edm_ctx *ctx, double *hbm_gbps, double *mfma_bf16_tflops, double *valu_fp32_tops);

/* Time-delay embedding, Section 2.1 step 1.
 * x   : float32 [L]
 * out : float32 [n][E], n = L - (E-1)*tau, out[p][j] = x[p + j*tau]. */
int edm_embed(edm_ctx *ctx, const float *x, int64_t L, int32_t E, int32_t tau,
              float *out);

/* All k-nearest-neighbour table of one library series, Section 2.1 step 2
 * and Algorithms 1-2 (distances and the k smallest per row, "Normalize D_k").
 * x    : float32 [L], L <= EDM_L_MAX
 * E    : 1..EDM_E_MAX;  k: 1..EDM_K_MAX, 0 means E+1
 * idx  : int32 [nq][k]  neighbour indices q, ascending by (key, q)   (required)
 * dist : float32 [nq][k] Euclidean distances, computed in float64  (or NULL)
 * w    : float32 [nq][k] simplex weights exp(-d_i/min d) / sum, Section 2.1
 *        step 3; when min d = 0 the weights are 1 at zero distance and 0
 *        elsewhere before normalising                               (or NULL)
 * nq = L - (E-1)*tau - Tp.
 * In EDM_FORM_CHOSEN with tau = 1, k = E+1, E >= 5, L <= 32000 and dist ==
 * NULL, the table comes from the matrix-core filtered scan (same result). */
int edm_knn(edm_ctx *ctx, const float *x, int64_t L, int32_t E, int32_t tau,
            int32_t Tp, int32_t k, int32_t *idx, float *dist, float *w);

/* Batched simplex lookup through one table, Section 2.1 step 3 and
 * Algorithm 3, with the Pearson skill of Section 2.1 step 4 computed on the
 * fly (Section 3.4).
 * idx, w : the table of edm_knn, int32/float32 [nq][k]
 * Y      : float32 [N][ldy] targets; row j must hold at least
 *          nq + (E-1)*tau + Tp samples (ldy >= that)
 * pred   : float32 [N][nq] predictions Yhat(p) = sum_i w_i Y[j][t(q_i)+Tp]
 *          (or NULL)
 * rho    : float32 [N] Pearson correlation of (Y[j][t(p)+Tp], Yhat(p)) over
 *          p in [0, nq); NaN when either is constant               (or NULL) */
int edm_lookup(edm_ctx *ctx, const int32_t *idx, const float *w, int64_t nq,
               int32_t k, int32_t E, int32_t tau, int32_t Tp, const float *Y,
               int64_t N, int64_t ldy, float *pred, float *rho);

/* Simplex embedding-dimension sweep: every series predicts itself Tp steps
 * ahead at E = 1..E_max with k = E+1 (Section 2.1: E is determined
 * empirically; Section 3.4 uses each target's optimal E).
 * X     : float32 [N][ldx];  L: (host) int64 [N] lengths, L[s] <= ldx
 * rho   : float32 [N][E_max]; NaN where E is infeasible for the series
 * E_opt : int32 [N], the smallest E attaining the largest non-NaN rho, or 0
 *         when no E is feasible.  E_max: 1..EDM_E_MAX. */
int edm_simplex_sweep(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N,
                      int64_t ldx, int32_t E_max, int32_t tau, int32_t Tp,
                      float *rho, int32_t *E_opt);

/* All-to-all convergent cross mapping (Section 2.1, all pairs; Section 3.4:
 * the library is embedded at the target's optimal E, targets are grouped by
 * E and each library's table is built once per E and reused).
 * X     : float32 [Nl][ldx] libraries, Lx: (host) int64 [Nl] lengths
 * Y     : float32 [Nt][ldy] targets,   Ly: (host) int64 [Nt] lengths
 * E_tgt : int32 [Nt] (device), 0..EDM_E_MAX; 0 marks a target without an E
 * rho   : float32 [Nl][Nt], rho[i][j] = skill of predicting Y_j from X_i.
 *         Pair (i, j) is defined iff E_tgt[j] >= 1, Ly[j] >= Lx[i] and the
 *         library is long enough for k = E_tgt[j]+1; Y_j is read on the
 *         library's time axis [0, Lx[i]).  Undefined pairs and constant
 *         series give NaN.  Tp = 0 is the paper's cross map. */
int edm_ccm(edm_ctx *ctx, const float *X, const int64_t *Lx, int64_t Nl,
            int64_t ldx, const float *Y, const int64_t *Ly, int64_t Nt,
            int64_t ldy, const int32_t *E_tgt, int32_t tau, int32_t Tp,
            float *rho);

/* Cross mapping on library subsamples: the convergence test of CCM (the
 * skill of a causal pair grows with the library size; the criterion Section
 * 2.1's method rests on, which the paper does not run).  Library x (float32
 * [L]) is embedded at E; subsample s is a set of candidate points, the host
 * int32 indices sets[set_off[s] .. set_off[s+1]), strictly ascending, in
 * [0, nq) with nq = L - (E-1)*tau - Tp.  Every query p in [0, nq) takes its
 * k = E+1 nearest neighbours inside the set (excluding |q - p| <= r, the
 * context's exclusion radius, and ties to the lower index), weights as
 * Section 2.1 step 3, and each target is predicted over all nq queries.
 * Y     : float32 [Nt][ldy] targets, ldy >= L, read on the library's time axis
 * sets, set_off : (host) int32 [set_off[S]], int64 [S+1] with set_off[0] = 0
 * idx   : int32 [S][nq][k] the subsamples' tables, or NULL
 * rho   : float32 [S][Nt], NaN where a side is constant
 * Every set needs at least k + 2r + 1 members (EDM_E_SHORT otherwise). */
int edm_ccm_subsample(edm_ctx *ctx, const float *x, int64_t L, const float *Y, int64_t Nt,
                      int64_t ldy, int32_t E, int32_t tau, int32_t Tp, const int32_t *sets,
                      const int64_t *set_off, int64_t S, int32_t *idx, float *rho);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as edm_simplex_sweep in EDM_FORM_PLAIN (one
 * fused scan per E, the context's exclusion radius), whatever the context's
 * form, with no allocation of any kind.  Its scratch (the lengths and the
 * per-block co-moments, 8 N + 48 N E_max ceil(L_max/256) bytes) lives in a
 * static device array of 64 MiB per GPU, resolved by edm_ctx_create and held
 * until the process ends; larger inputs return EDM_E_NOMEM (use
 * edm_simplex_sweep).  Every call on a GPU shares that array: calls that
 * overlap in time on one GPU (several contexts or threads) race.  With equal
 * lengths the call makes no host-to-device copy; otherwise L is copied from
 * the caller's host array.  Kernel timing (edm_ctx_set_timing) does not
 * cover this call. */
int edm_simplex_sweep_noalloc(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N,
                              int64_t ldx, int32_t E_max, int32_t tau, int32_t Tp,
                              float *rho, int32_t *E_opt);

/* The method's pipeline in one call (Section 3.4): the simplex E sweep of
 * every series (Tp = 1, E = 1..E_max) picks each series' E*, then every
 * ordered pair is cross-mapped at the target's E* (Tp = 0), the series being
 * both the libraries and the targets.  Results equal edm_simplex_sweep
 * followed by edm_ccm with E_tgt = E_opt and Tp = 0.
 * In EDM_FORM_CHOSEN with tau = 1 (and the sweep's lists of every E fitting
 * the workspace limit) the cross map's tables are derived from the sweep's:
 * at dimension E the Tp = 0 candidates are the Tp = 1 candidates plus the
 * point m1 = L - E, so a query's table is its sweep list with that point
 * offered last, and only query m1 needs a scan.  The targets are grouped by
 * E* on the device: the call never synchronises the stream, and with equal
 * lengths it makes no host-to-device copy either, so it can be captured in a
 * HIP graph (after one uncaptured call has grown the workspace).
 * X       : float32 [N][ldx] series, lengths L (host) [N]
 * rho_sweep, E_opt : as edm_simplex_sweep
 * rho     : float32 [N][N], rho[i][j] = library i, target j; NaN where the
 *           pair is undefined (L[j] < L[i], E_opt[j] = 0, a constant side). */
int edm_sweep_ccm(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N, int64_t ldx,
                  int32_t E_max, int32_t tau, float *rho_sweep, int32_t *E_opt, float *rho);

/* ---------------------------------------------------------------------------
 * Batched CCM plan: libraries of uneven length and targets of uneven E in
 * one graph of persistent launches (Section 3.4's grouping by E, batched over
 * libraries).  The plan is built once from the host lengths and E values:
 * libraries are ordered longest first and split into batches that fit the
 * workspace limit; per batch, one persistent kernel per E group builds every
 * table the library's targets need (one candidate scan per group, as the
 * chosen form of edm_ccm) and one persistent kernel per E runs the lookups,
 * each lookup item a group of up to 16 libraries against one staged tile of
 * targets.  Work items are pulled from device counters, longest first.  The whole
 * sequence is captured into a HIP graph on the first edm_ccm_plan_run and
 * replayed afterwards (re-captured when the buffers change; a context on the
 * legacy default stream enqueues the launches directly instead, since that
 * stream cannot be captured).  Results equal edm_ccm bit for bit.  tau = 1.
 * The form is the context's at edm_ccm_plan_create: in EDM_FORM_CHOSEN the
 * tables of E >= 5 of libraries up to 32000 samples come from the matrix-core
 * filtered scan (same tables), and the plan holds that filter's norm arrays
 * for every library (Nl x 16 x ~L_max x 4 bytes).
 * ------------------------------------------------------------------------- */
typedef struct edm_plan edm_plan;

/* Launch shapes of a plan (chosen by an autotuner; see edm_tune_default). */
typedef struct {
  int32_t tables_wg_per_cu;   /* 0: one workgroup per table item; >0: persistent workgroups per CU */
  int32_t lookup_wg_per_cu;   /* 0: one workgroup per lookup item; >0: persistent workgroups per CU */
  int32_t lookup_targets;     /* targets staged per lookup item, 1..16 (fewer where the
                                 longest library's window would pass 160 KB of LDS) */
  int32_t filter_stride;      /* chosen form: the matrix-core filter's first pass visits one
                                 candidate tile in filter_stride (1..8), which bounds each
                                 query's k-th key; 0: by E group and series length.  Tables
                                 and rho do not depend on it, only the time. */
} edm_tune;

void edm_tune_default(edm_tune *tune);

/* Build a plan.  Lx (host) int64 [Nl], Ly (host) int64 [Nt], E_tgt (host)
 * int32 [Nt] in 0..20 (0: no E, the column stays NaN); ldx, ldy the row
 * strides the run will use; tune may be NULL (defaults).  Allocates the
 * plan's device memory (work lists, offsets, one batch of tables and, in the
 * chosen form, the filter's per-library norms). */
int edm_ccm_plan_create(edm_ctx *ctx, const int64_t *Lx, int64_t Nl, int64_t ldx,
                        const int64_t *Ly, int64_t Nt, int64_t ldy, const int32_t *E_tgt,
                        int32_t Tp, const edm_tune *tune, edm_plan **plan);

/* Run (replay) the plan on X [Nl][ldx], Y [Nt][ldy] into rho [Nl][Nt], with
 * the same definition of defined pairs as edm_ccm. */
int edm_ccm_plan_run(edm_ctx *ctx, edm_plan *plan, const float *X, const float *Y, float *rho);

/* Release the plan (waits for the context's stream first if ctx != NULL). */
void edm_ccm_plan_destroy(edm_ctx *ctx, edm_plan *plan);

/* ---------------------------------------------------------------------------
 * Learned embedding-dimension surrogate.
 *
 * A small 1-D convolutional network predicts a series' optimal E from the
 * series itself; it is trained on the E* that edm_simplex_sweep selects (the
 * method's own E selection: Section 2.1 step 1 leaves E to be determined
 * empirically and Section 3.4 uses each target's optimal E).  Network:
 * conv(1->C, EDM_NET_KW) -> ReLU -> conv(C->C) -> ReLU -> conv(C->C) -> ReLU
 * -> mean over time -> linear(C->20), zero "same" padding.  Parameters are one
 * float32 device array of edm_net_param_count(C) values laid out as
 * w1[C][1][KW], b1[C], w2[C][C][KW], b2[C], w3[C][C][KW], b3[C], wo[20][C],
 * bo[20].  C: 1..64.  Series are z-scored float32 rows X[B][ldx], length L.
 * ------------------------------------------------------------------------- */
#define EDM_NET_KW 7
#define EDM_NET_CLASSES 20
#define EDM_NET_C_MAX 64

/* Number of float32 parameters of the network with C channels (host only). */
int64_t edm_net_param_count(int32_t C);

/* Forward pass: logits[B][20] (float32, device); class c is E = c + 1. */
int edm_net_forward(edm_ctx *ctx, const float *params, int32_t C, const float *X, int64_t B,
                    int64_t L, int64_t ldx, float *logits);

/* Inference form of edm_net_forward: the two C -> C convolutions run on the
 * BF16 matrix cores (inputs and weights rounded to BF16, FP32 accumulation);
 * layer 1, pooling and the linear layer stay float32.  C must be 32 or 64.
 * Training uses edm_net_loss_grad (float32 throughout). */
int edm_net_forward_bf16(edm_ctx *ctx, const float *params, int32_t C, const float *X, int64_t B,
                         int64_t L, int64_t ldx, float *logits);

/* Mean softmax cross-entropy of the batch against labels[B] (int32 E in
 * 1..20, device) and its gradient with respect to the parameters.
 * loss: float32 scalar (device); grad: float32 [edm_net_param_count(C)]. */
int edm_net_loss_grad(edm_ctx *ctx, const float *params, int32_t C, const float *X,
                      const int32_t *labels, int64_t B, int64_t L, int64_t ldx, float *loss,
                      float *grad);

/* One Adam step (Kingma & Ba) in place: m, v are the moment buffers of the
 * same length n, step >= 1 counts updates (bias correction). */
int edm_net_adam(edm_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n,
                 int32_t step, float lr, float beta1, float beta2, float eps);

/* E selection driven by the network: for every series s the candidate set
 * is the m_top classes with the largest logits; if the largest softmax
 * probability is below min_conf the candidate set is every E in 1..E_max
 * (the plain sweep, as fallback).  The simplex skill (Tp ahead, k = E+1, the
 * same computation as edm_simplex_sweep) is evaluated at the candidates only
 * and E_opt[s] is the smallest E with the largest non-NaN rho among them.
 * logits: float32 [N][20] (device); rho: float32 [N][E_max] (device), NaN
 * where E was not evaluated or is infeasible; E_opt: int32 [N] (device);
 * n_fallback (host, or NULL): number of series that took the full sweep.
 * In EDM_FORM_CHOSEN and EDM_FORM_BATCHED (tau = 1, no exclusion radius)
 * the series with every E to evaluate run the batched sweep (their rows are
 * packed in the workspace); the others one exact scan per candidate E.
 * Synchronises the stream once (the candidate sets are read back). */
int edm_select_E(edm_ctx *ctx, const float *X, const int64_t *L, int64_t N, int64_t ldx,
                 int32_t E_max, int32_t tau, int32_t Tp, const float *logits, int32_t m_top,
                 float min_conf, float *rho, int32_t *E_opt, int64_t *n_fallback);

#ifdef __cplusplus
}
#endif

#endif /* EDM_H */
