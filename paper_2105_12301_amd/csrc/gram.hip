// Chosen form of the distance step for E >= 5: a BF16 matrix-core Gram
// filter with an exact re-rank (kEDM paper: Section 2.1 steps 1-4 and
// Algorithms 1-2 define what is computed; the filter is this library's own
// design for gfx950).
//
// Arithmetic
// ----------
// With centred samples b = x - mu (mu: one float32 constant per series), the
// squared distance of query p and candidate q at dimension E is
//     N_E(p) + N_E(q) - 2 G_E(p, q),
// N_E the squared norm of a point's E samples and G_E their lag-wise dot
// product.  G is a matrix product over the lag index, so the matrix cores
// evaluate it for a 32 x 32 tile of (candidate, query) pairs per
// v_mfma_f32_32x32x16_bf16.  Each centred sample is split into two BF16
// numbers, b = hi + lo + r with |r| <= 2^-16 |b|, and hi*hi' + hi*lo' + lo*hi'
// (three MFMAs, FP32 accumulation) gives G with an error below
// 6.1 * 2^-16 |v_p| |v_q| plus the FP32 accumulation error.  Two more slots
// of the contraction finish the test inside the chain: the candidate's norm
// (operand one on the query side) and the query's threshold (operand one on
// the candidate side, -T as a BF16 pair rounded down), so one chain yields
//     e = s N_E(q) - 2 G_E(p, q) - T',   s = 1 - 2^-12,  T' >= T,
//     T = kth_E(p) - s N_E(p) + 2^-90.
// e < 0 holds for every candidate whose exact key is at most the query's
// current k-th key: the slack 2^-12 (N_E(p) + N_E(q)) is at least three times
// every rounding above (the canonical key's own rounding, the centring and
// the threshold's rounding included).  A candidate with e >= 0 cannot enter
// the list.  Every candidate with e < 0 ("survivor") is re-ranked with the
// exact float32 key of Algorithm 1 (lag order, one rounding per operation,
// contraction off) and offered to the same sorted register lists as the
// exact scan, so the tables and correlations are bit-identical to the exact
// scan's.  |T| is capped at 2^120 (finite operands) and a series with
// |x - mu| above 2^56 switches the filter off (every candidate survives).
//
// Layout on the chip
// ------------------
// * Grid: workgroups are dispatched round-robin over the 8 dies (one L2
//   each); the query blocks of one series are mapped to one die, so its
//   samples and norms are fetched into one L2 and shared there.
// * Workgroup = 8 waves = the 256 queries of one exact-scan block; LDS holds
//   the BF16 hi and lo halves of the centred series (matrix operands), the
//   float32 series (exact re-rank, weights) up to kGramLdsXsMax samples
//   (beyond, the XG instantiation reads it from global memory), and one
//   survivor queue per lane.
// * A wave owns 32 queries.  MFMA operand A holds 32 candidates (tile rows),
//   operand B the wave's 32 queries (tile columns, fixed between threshold
//   updates), so lane l ends with the 16 estimates of candidates
//   8(v/4) + 4(l/32) + v%4 for query l%32.  The two lanes of a query (l and
//   l+32) keep top-k lists over their own half of the candidates, each in
//   ascending q, merged by a bitonic network at the end.
// * K-slots: lags 0..E_hi-1, one norm slot per E of the group, the threshold
//   slot, zeros; a group that does not fit one 16-slot chunk shares a first
//   chunk of lags 0..S-1 (S = min(E_lo, 16)) and keeps one chunk per E.
// * Two passes over the candidate tiles.  Pass 1 visits every tile, or one
//   in three or four (BF16 hi halves only, one product per chunk) and keeps, per lane and value
//   slot, the candidate with the smallest hi*hi estimate at E_hi (one in
//   m/32: the bound is near the true k-th key, so few candidates survive
//   pass 2 before the lists fill); the exact keys of a query's 32 slot winners bound
//   its final k-th key for every E of the group.  Pass 2 tests every tile:
//   the OR over E of the estimates' sign bits is a per-lane mask, queued with
//   the tile index in LDS without a branch; the queue is re-ranked when some
//   lane holds kQueueCap masks, and at the end, and each re-rank refreshes the
//   thresholds with min(bound, K-th key of the query's two half-lists).
#include <cstdint>
#include <type_traits>

#include "../../include/edm.h"
#include "device_common.h"
#include "kernels.h"
#include "scan_common.h"

#pragma clang fp contract(off)

namespace edm {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kGramWaves = 8;
constexpr int kGramThreads = kGramWaves * kWave;
static_assert(kGramWaves * 32 == kKnnThreads, "a workgroup covers one query block of the exact scan");
constexpr float kGramScale = 1.0f - 0x1p-12f;  // s = 1 - 2^-12
constexpr float kGramFloor = 0x1p-90f;          // absolute slack: flushed tiny products
constexpr float kGramSafeMax = 0x1p56f;         // larger |x - mu| switches the filter off
constexpr int kP1Tiles = 4;                     // pass-1 tiles per step
constexpr int kQueueCap = 16;                   // queued tile masks per lane before a re-rank
constexpr int kGramXcds = 8;                    // accelerator dies (one L2 each), round-robin dispatch
constexpr float kGramBig = 0x1p120f;            // |threshold| cap: finite BF16 operands
constexpr int kBufWord3 = 0x00020000;           // raw buffer resource, dword 3 (GFX9 family)

__device__ __forceinline__ uint32_t bf16_bits(float f) {  // round to nearest even (finite f)
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }
// hi | lo << 16 with v = hi + lo to 2^-16 relative.
__device__ __forceinline__ uint32_t split_pack(float v) {
  const uint32_t hi = bf16_bits(v);
  return hi | (bf16_bits(v - bf16_val(hi)) << 16);
}
__device__ __forceinline__ float unpack_sum(uint32_t w) {
  return bf16_val(w & 0xffffu) + bf16_val(w >> 16);
}
// Both BF16 halves of a word times -2 (exact).
__device__ __forceinline__ uint32_t scale_m2(uint32_t w) {
  return bf16_bits(-2.0f * bf16_val(w & 0xffffu)) | (bf16_bits(-2.0f * bf16_val(w >> 16)) << 16);
}

// Eight consecutive BF16 values starting at element `base` of a 16-bit array
// viewed as words: aligned word reads and a funnel shift for odd starts.
__device__ __forceinline__ void read_window(const uint32_t *__restrict__ w32, int base,
                                            uint32_t (&out)[4]) {
  const int w0 = base >> 1;
  const uint32_t sh = static_cast<uint32_t>(base & 1) * 16u;
  uint32_t W[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) W[i] = w32[w0 + i];
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = __builtin_amdgcn_alignbit(W[i + 1], W[i], sh);
}

// Minimum of two floats as the median of (a, b, -inf): one instruction and
// no NaN canonicalisation (the operands are finite or +inf).
__device__ __forceinline__ float min2(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, -__builtin_inff());
}

// e with its 10 low mantissa bits replaced by t (t < 1024).
__device__ __forceinline__ float with_low10(float e, uint32_t t) {
  return __uint_as_float((__float_as_uint(e) & 0xfffffc00u) | t);
}

// Ascending bitonic sort of 16 values held in registers.
__device__ __forceinline__ void sort16(float (&a)[16]) {
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const float x = a[i], y = a[l];
          const bool up = (i & k) == 0;
          a[i] = up ? fminf(x, y) : fmaxf(x, y);
          a[l] = up ? fmaxf(x, y) : fminf(x, y);
        }
      }
}

// Largest value of v over the wave (butterfly over the 64 lanes).
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v = max(v, __shfl_xor(v, m));
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ f32x16_t mfma(const uint32_t (&a)[4], const uint32_t (&b)[4],
                                         f32x16_t c) {
  const u32x4_t av = {a[0], a[1], a[2], a[3]};
  const u32x4_t bv = {b[0], b[1], b[2], b[3]};
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                 __builtin_bit_cast(bf16x8_t, bv), c, 0, 0, 0);
}

// K-slot layout of a group [ELO, EHI].  The last chunk ends with one norm
// slot per E of the group and one threshold slot; a group whose lags, norms
// and threshold do not fit one 16-slot chunk uses a shared first chunk of
// lags 0..S-1 (S <= ELO, the same for every E of the group).
template <int ELO, int EHI>
struct Layout {
  static constexpr int kLo = ELO;
  static constexpr int NG = EHI - ELO + 1;
  static constexpr bool kShared = EHI + NG + 1 > 16;
  static constexpr int S = kShared ? (ELO < 16 ? ELO : 16) : 0;  // lags of the shared chunk
  static constexpr int kChunks = kShared ? 2 : 1;
  static constexpr int kFirst = kShared ? 1 : 0;  // first chunk that depends on E
  static constexpr int kLast = kChunks - 1;
  static constexpr int kNorm = EHI - S;           // first norm slot of the last chunk
  static constexpr int kT = kNorm + NG;           // threshold slot of the last chunk
  static_assert(ELO >= kGramEMin && EHI <= EDM_E_MAX && ELO <= EHI, "E range");
  static_assert(kT < 16, "E range does not fit the slot layout");
  // Lag held by slot s of chunk C (-1: not a lag slot).
  static constexpr int lag(int C, int s) {
    if (kShared && C == 0) return s < S ? s : -1;
    return s < kNorm ? S + s : -1;
  }
  // 0: zero, 1: lag, 2 + g: norm of E = ELO + g, 2 + NG: threshold
  static constexpr int kind(int C, int s) {
    if (lag(C, s) >= 0) return 1;
    if (C != kLast) return 0;
    if (s >= kNorm && s < kT) return 2 + (s - kNorm);
    return s == kT ? 2 + NG : 0;
  }
  static constexpr int first_lag(int C) { return (kShared && C == 1) ? S : 0; }
};

// Candidate-side words of chunk C: lane half h1 holds slots 8 h1 .. 8 h1 + 7.
// wh/wl: the window of samples first_lag(C) + 8 h1 .. + 7 of the candidate.
template <class Lay, int C>
__device__ __forceinline__ void build_a(uint32_t (&ah)[4], uint32_t (&al)[4],
                                        const uint32_t (&wh)[4], const uint32_t (&wl)[4],
                                        const uint32_t (&nr)[Lay::NG], bool h1) {
  constexpr uint32_t kOne = 0x3f80u;  // BF16 1.0
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t vh[2], vl[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      uint32_t h = 0, l = 0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = Lay::kind(C, 8 * hh + 2 * w + u);
        const int sh = 16 * u;
        const uint32_t m = 0xffffu << sh;
        if (k == 1) {
          h |= wh[w] & m;
          l |= wl[w] & m;
        } else if (k >= 2 && k < 2 + Lay::NG) {
          h |= (nr[k - 2] & 0xffffu) << sh;
          l |= (nr[k - 2] >> 16) << sh;
        } else if (k == 2 + Lay::NG) {
          h |= kOne << sh;
        }
      }
      vh[hh] = h;
      vl[hh] = l;
    }
    ah[w] = h1 ? vh[1] : vh[0];
    al[w] = h1 ? vl[1] : vl[0];
  }
}

// Query-side words of chunk C for dimension E: lags below E (already scaled
// by -2), one in E's norm slot (hi operand only), zeros elsewhere; the
// threshold slot is written by set_threshold.
template <class Lay, int C, int E>
__device__ __forceinline__ void build_b(uint32_t (&bh)[4], uint32_t (&bl)[4],
                                        const uint32_t (&qh)[4], const uint32_t (&ql)[4],
                                        bool h1) {
  constexpr uint32_t kOne = 0x3f80u;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t vh[2], vl[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      uint32_t h = 0, l = 0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int s = 8 * hh + 2 * w + u;
        const int k = Lay::kind(C, s);
        const uint32_t m = u ? 0xffff0000u : 0xffffu;
        if (k == 1 && Lay::lag(C, s) < E) {
          h |= qh[w] & m;
          l |= ql[w] & m;
        } else if (k == 2 + (E - Lay::kLo)) {
          h |= u ? (kOne << 16) : kOne;
        }
      }
      vh[hh] = h;
      vl[hh] = l;
    }
    bh[w] = h1 ? vh[1] : vh[0];
    bl[w] = h1 ? vl[1] : vl[0];
  }
}

// BF16 bits of f rounded toward -inf (finite f).
__device__ __forceinline__ uint32_t bf16_bits_down(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t t = u >> 16;
  return ((u & 0x80000000u) && (u & 0xffffu)) ? t + 1u : t;
}

// Threshold slot of a query operand: -T as hi + lo with hi + lo <= -T, so the
// product chain yields D - T' with T' >= T (never fewer survivors).
template <class Lay>
__device__ __forceinline__ void set_threshold(uint32_t (&bh)[4], uint32_t (&bl)[4], float T,
                                              bool h1) {
  constexpr int s = Lay::kT;
  constexpr int w = (s & 7) >> 1;
  constexpr int sh = 16 * (s & 1);
  constexpr uint32_t m = 0xffffu << sh;
  const float u = -T;
  const uint32_t hi = bf16_bits(u);
  const uint32_t lo = bf16_bits_down(u - bf16_val(hi));
  if (h1 == ((s >> 3) != 0)) {
    bh[w] = (bh[w] & ~m) | (hi << sh);
    bl[w] = (bl[w] & ~m) | (lo << sh);
  }
}

// Sign bits of 16 estimates, value v = 4 j + b at bit 8 j + 4 + b (so the
// lowest set bit is the lowest candidate); bits 0-3 of every byte are zero.
__device__ __forceinline__ uint32_t sign_mask(const uint32_t (&e)[16]) {
  uint32_t d[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    // bytes: top byte of e[b], e[4 + b] | e[8 + b], e[12 + b]
    const uint32_t p0 = __builtin_amdgcn_perm(e[4 + b], e[b], 0x0c0c0703u);
    const uint32_t p1 = __builtin_amdgcn_perm(e[12 + b], e[8 + b], 0x0c0c0703u);
    d[b] = __builtin_amdgcn_perm(p1, p0, 0x05040100u);  // byte j: value 4 j + b
  }
  return (d[3] & 0x80808080u) | ((d[2] >> 1) & 0x40404040u) | ((d[1] >> 2) & 0x20202020u) |
         ((d[0] >> 3) & 0x10101010u);
}
constexpr uint32_t kSignBits = 0xf0f0f0f0u;

// Tile index spread over the low nibbles of the first three bytes.
__device__ __forceinline__ uint32_t tile_code(uint32_t t) {
  return (t & 15u) | ((t & 0xf0u) << 4) | ((t & 0xf00u) << 8);
}
__device__ __forceinline__ uint32_t tile_of(uint32_t code) {
  return (code & 15u) | ((code >> 4) & 0xf0u) | ((code >> 8) & 0xf00u);
}

// (key, index) order with the index compared unsigned (index -1 sorts last).
__device__ __forceinline__ bool lex_less(float ka, int ia, float kb, int ib) {
  return ka < kb || (ka == kb && static_cast<uint32_t>(ia) < static_cast<uint32_t>(ib));
}

// Final step (Section 2.1 step 3) for dimension E of query p, E one of E0
// and E1 = E0 + 1 (or E0 alone when E1 == E0): the same float64 arithmetic,
// in the same order, as finish_list, with the lag and neighbour counts set
// at run time so that the two lane halves finish two dimensions at once.
// idx: the sorted list (E + 1 entries used); the query's samples come from xs
// (LDS or global: every index read here lies inside the series).
template <int E0, int E1>
__device__ __forceinline__ Mom finish_round(const KnnArgs &a, int row, int p, int L, int Tp,
                                            uint32_t need, const int (&idx)[E1 + 1], int E,
                                            const float *__restrict__ xs) {
  constexpr int KM = E1 + 1;
  const bool hi = E != E0;
  const int K = E + 1;
  const int mE = L - (E - 1) - Tp;
  Mom mine = mom_zero();
  const bool want_table = a.mom == nullptr && ((need >> (E - 1)) & 1u);
  if (p < mE && mE - 1 >= K && (a.mom != nullptr || want_table)) {
    int q[KM];
    double D[KM];
    double dmin = __builtin_inf();
#pragma unroll
    for (int r = 0; r < KM; ++r) {
      q[r] = idx[r] < 0 ? 0 : idx[r];
      double s2 = 0.0;
#pragma unroll
      for (int j = 0; j < E1; ++j) {
        if (j < E0 || hi) {
          const double d = static_cast<double>(xs[p + j]) - static_cast<double>(xs[q[r] + j]);
          s2 += d * d;
        }
      }
      D[r] = sqrt(s2);
      if (r < KM - 1 || hi || E1 == E0) dmin = fmin(dmin, D[r]);
    }
    double wsum = 0.0;
#pragma unroll
    for (int r = 0; r < KM; ++r) {
      const double d = D[r];
      const double wq = dmin > 0.0 ? exp(-d / dmin) : (d == 0.0 ? 1.0 : 0.0);
      if (r < KM - 1 || hi || E1 == E0) wsum += wq;
      D[r] = wq;
    }
    const double inv = 1.0 / wsum;
    if (want_table) {
      int32_t *ti;
      float *tw;
      int64_t base;
      if (a.tbl_off) {
        const int64_t o = a.tbl_off[static_cast<int64_t>(row) * (EDM_E_MAX + 1) + E];
        ti = a.tbl_idx + o;
        tw = a.tbl_w + o;
        base = static_cast<int64_t>(p) * K;
      } else {
        ti = hi ? a.idxE[E1] : a.idxE[E0];
        tw = hi ? a.wE[E1] : a.wE[E0];
        base = static_cast<int64_t>(row) * (hi ? a.strideE[E1] : a.strideE[E0]) +
               static_cast<int64_t>(p) * K;
      }
#pragma unroll
      for (int i = 0; i < KM; ++i) {
        if (i < KM - 1 || hi || E1 == E0) {
          ti[base + i] = q[i];
          tw[base + i] = static_cast<float>(D[i] * inv);
        }
      }
    } else {
      int32_t *keep = hi ? a.keepE[E1] : a.keepE[E0];
      if (keep) {  // sweep mode: keep the sorted list (and weights) for a later cross map
        const int64_t ko = static_cast<int64_t>(row) * (hi ? a.keep_strideE[E1] : a.keep_strideE[E0]) +
                           static_cast<int64_t>(p) * K;
        float *keepw = hi ? a.keepWE[E1] : a.keepWE[E0];
#pragma unroll
        for (int i = 0; i < KM; ++i)
          if (i < KM - 1 || hi || E1 == E0) keep[ko + i] = q[i];
        if (keepw) {
#pragma unroll
          for (int i = 0; i < KM; ++i)
            if (i < KM - 1 || hi || E1 == E0) keepw[ko + i] = static_cast<float>(D[i] * inv);
        }
      }
      const int o_off = (E - 1) + Tp;
      double yh = 0.0;
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (i < KM - 1 || hi || E1 == E0) yh += (D[i] * inv) * static_cast<double>(xs[q[i] + o_off]);
      mine.n = 1.0;
      mine.mo = static_cast<double>(xs[p + o_off]);
      mine.mp = yh;
    }
  }
  return mine;
}

// One workgroup's share of a filtered scan: query block `bx` of row `row`,
// every E in [ELO, EHI].  Same outputs as the exact group scan.
// XG: the exact float32 samples are read from global memory (L2) instead of
// an LDS copy, which leaves room in LDS for series up to kGramLMax.
template <int ELO, int EHI, bool XG>
__device__ __forceinline__ void gram_scan(const KnnArgs &a, const int row, const int bx,
                                          float *__restrict__ smem) {
  using Lay = Layout<ELO, EHI>;
  constexpr int NG = Lay::NG;
  constexpr int TOT = list_off<ELO>(EHI + 1);
  constexpr int NCH = Lay::kChunks;
  constexpr int C0 = Lay::kFirst;
  __shared__ Mom wmom[kGramWaves][NG];
  const uint32_t need = a.need_dev ? a.need_dev[row] : a.need;
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int L = static_cast<int>(a.L_dev ? a.L_dev[row] : a.L_uni);
  const int Tp = a.Tp;
  const int m_lo = L - (ELO - 1) - Tp;  // queries = candidates at ELO, the widest range
  if (m_lo - 1 < ELO + 1) return;
  const int blk0 = bx * kKnnThreads;
  if (blk0 >= m_lo) return;

  const int64_t ld = a.gram_ld;                            // norm rows
  const int64_t lds = a.gram_lds > 0 ? a.gram_lds : ld;   // LDS rows (>= L + kGramPad)
  float *xs = smem;  // unused when XG
  uint16_t *xh = reinterpret_cast<uint16_t *>(XG ? smem : smem + lds);
  uint16_t *xl = xh + lds;
  // exact samples: LDS copy (zero past L), or the global row through a
  // buffer resource of L samples (the hardware returns zero past L; those
  // reads only feed keys that are discarded)
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(x), static_cast<short>(0), L * static_cast<int>(sizeof(float)), kBufWord3);
  auto xat = [&](int i) -> float {
    if constexpr (XG) {
      const int off = i * static_cast<int>(sizeof(float));
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off, 0, 0));
    } else {
      return xs[i];
    }
  };
  const uint32_t *xh32 = reinterpret_cast<const uint32_t *>(xh);
  const uint32_t *xl32 = reinterpret_cast<const uint32_t *>(xl);
  uint32_t *qbuf_all = reinterpret_cast<uint32_t *>(xl + lds);  // [wave][kQueueCap][64] queues
  const float mu = a.gram_mu[row];
  const uint32_t *__restrict__ nrm =
      a.gram_nrm + (static_cast<int64_t>(row) * kGramNE + (ELO - kGramEMin)) * ld;

  bool bad = false, big = false;
  for (int i = threadIdx.x; i < L + kGramPad; i += kGramThreads) {
    float v = 0.0f, b = 0.0f;
    if (i < L) {
      v = x[i];
      bad |= !isfinite(v);
      b = v - mu;
    }
    big |= !(fabsf(b) <= kGramSafeMax);
    if constexpr (!XG) xs[i] = v;
    const uint32_t pk = split_pack(b);
    xh[i] = static_cast<uint16_t>(pk & 0xffffu);
    xl[i] = static_cast<uint16_t>(pk >> 16);
  }
  if (bad) atomicOr(a.status, 1);
  const bool unsafe = __syncthreads_or(big);

  const int lane = threadIdx.x & (kWave - 1);
  const int n = lane & 31;
  const bool h1 = lane >= 32;
  const int wave = threadIdx.x / kWave;
  const int pw = __builtin_amdgcn_readfirstlane(blk0 + 32 * wave);
  const int p = pw + n;
  const bool qry = p < m_lo;
  const int pc = qry ? p : 0;


  // Lists of E that are not needed (or whose range ends before p) stay idle.
  auto list_active = [&](int E) {
    return p < L - (E - 1) - Tp && (a.mom != nullptr || ((need >> (E - 1)) & 1u));
  };
  bool act_any = false;
  static_for<ELO, EHI>([&](auto EC) { act_any = act_any || list_active(decltype(EC)::value); });

  // Query norms s N_E(p); T_E = kth_E - s N_E(p) rides in the threshold slot.
  float nq[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) nq[g] = unpack_sum(nrm[g * ld + pc]);

  // Query operands (fixed between threshold updates).
  uint32_t bsh[4], bsl[4];
  uint32_t bh[NG][NCH - C0][4], bl[NG][NCH - C0][4];
  static_for<0, NCH - 1>([&](auto CC) {
    constexpr int C = decltype(CC)::value;
    uint32_t qh[4], ql[4];
    read_window(xh32, pc + Lay::first_lag(C) + (h1 ? 8 : 0), qh);
    read_window(xl32, pc + Lay::first_lag(C) + (h1 ? 8 : 0), ql);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      qh[w] = scale_m2(qh[w]);
      ql[w] = scale_m2(ql[w]);
    }
    if constexpr (Lay::kShared && C == 0) {
      build_b<Lay, 0, EHI>(bsh, bsl, qh, ql, h1);
    } else {
      static_for<ELO, EHI>([&](auto EC) {
        constexpr int E = decltype(EC)::value;
        build_b<Lay, C, E>(bh[E - ELO][C - C0], bl[E - ELO][C - C0], qh, ql, h1);
      });
    }
  });

  // Candidate operands of the tile starting at c0 (A rows: candidates
  // c0 .. c0+31) and the shared chunk's partial products.
  // The candidate norms come from global memory: they are loaded one tile
  // ahead (fetch) so the load latency overlaps the current tile's work.
  uint32_t ah[NCH][4], al[NCH][4];
  f32x16_t acc_s = {};
  uint32_t nr[NG], nr_next[NG];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int g = 0; g < NG; ++g) nr_next[g] = nrm[g * ld + c0 + n];
  };
  // The LDS words of the next tile's windows are read one tile ahead as
  // well (rh, rl: five words per window; the funnel shift comes at use).
  uint32_t rh[NCH][5], rl[NCH][5];
  auto read_raw = [&](int c0) {
    static_for<0, NCH - 1>([&](auto CC) {
      constexpr int C = decltype(CC)::value;
      const int w0 = (c0 + n + Lay::first_lag(C) + (h1 ? 8 : 0)) >> 1;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        rh[C][i] = xh32[w0 + i];
        rl[C][i] = xl32[w0 + i];
      }
    });
  };
  auto load_tile = [&](int c0, int c_next) {
    const int cn = c_next < m_lo ? c_next : c0;  // in bounds: c0 < m_lo and gram_ld >= L + 64
#pragma unroll
    for (int g = 0; g < NG; ++g) nr[g] = nr_next[g];
    fetch(cn);
    static_for<0, NCH - 1>([&](auto CC) {
      constexpr int C = decltype(CC)::value;
      const uint32_t sh = static_cast<uint32_t>((n + Lay::first_lag(C)) & 1) * 16u;  // c0 is even
      uint32_t wh[4], wl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        wh[i] = __builtin_amdgcn_alignbit(rh[C][i + 1], rh[C][i], sh);
        wl[i] = __builtin_amdgcn_alignbit(rl[C][i + 1], rl[C][i], sh);
      }
      build_a<Lay, C>(ah[C], al[C], wh, wl, nr, h1);
    });
    read_raw(cn);
    acc_s = f32x16_t{};
    if constexpr (Lay::kShared) {
      acc_s = mfma(ah[0], bsh, acc_s);
      acc_s = mfma(ah[0], bsl, acc_s);
      acc_s = mfma(al[0], bsh, acc_s);
    }
  };
  auto estimate = [&](int g) {
    f32x16_t acc = acc_s;
#pragma unroll
    for (int C = C0; C < NCH; ++C) {
      acc = mfma(ah[C], bh[g][C - C0], acc);
      acc = mfma(ah[C], bl[g][C - C0], acc);
      acc = mfma(al[C], bh[g][C - C0], acc);
    }
    return acc;
  };
  // Exact float32 keys of candidate q for every E of the group (Algorithm 1,
  // one running sum); +inf where q is not a candidate of that E.
  auto exact_keys = [&](int q, bool ok, float (&key)[NG]) {
    float acc = 0.0f;
    static_for<0, EHI - 1>([&](auto JC) {
      constexpr int j = decltype(JC)::value;
      const float d = xat(pc + j) - xat(q + j);
      acc = acc + d * d;
      if constexpr (j + 1 >= ELO) {
        constexpr int E = j + 1;
        key[E - ELO] = (ok && q < L - (E - 1) - Tp) ? acc : __builtin_inff();
      }
    });
  };
  // The same for two candidates at once (two independent sums).
  auto exact_keys2 = [&](int q0, bool ok0, float (&k0)[NG], int q1, bool ok1, float (&k1)[NG]) {
    float a0 = 0.0f, a1 = 0.0f;
    static_for<0, EHI - 1>([&](auto JC) {
      constexpr int j = decltype(JC)::value;
      const float xp = xat(pc + j);
      const float d0 = xp - xat(q0 + j);
      const float d1 = xp - xat(q1 + j);
      a0 = a0 + d0 * d0;
      a1 = a1 + d1 * d1;
      if constexpr (j + 1 >= ELO) {
        constexpr int E = j + 1;
        k0[E - ELO] = (ok0 && q0 < L - (E - 1) - Tp) ? a0 : __builtin_inff();
        k1[E - ELO] = (ok1 && q1 < L - (E - 1) - Tp) ? a1 : __builtin_inff();
      }
    });
  };

  // Pass 1 (estimates only): lane v-slot b keeps the candidate with the
  // smallest estimate at E_hi (hi halves only, one product per chunk) among
  // the candidates 32 t + m(b); the 32 winners of
  // a query (16 per lane) are distinct candidates, so the K-th smallest of
  // their exact keys bounds the query's final K-th key from above, for every
  // E of the group.  These bounds cap the thresholds of pass 2 from the start.
  float ub[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) ub[g] = __builtin_inff();
  if (pw < m_lo) {
    // The tile index replaces the 10 low mantissa bits of the estimate (a
    // relative change below 2^-13: the ranking only picks candidates), so one
    // minimum keeps the estimate and its tile.  The estimates are finite.
    static_assert(kGramLMax / 32 <= 0x3ff, "tile index field");
    float bm[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) bm[v] = __builtin_inff();
    auto hi_tile = [&](int c0, const uint32_t (&nrv)[NG]) {
      uint32_t a_h[NCH][4];
      static_for<0, NCH - 1>([&](auto CC) {
        constexpr int C = decltype(CC)::value;
        uint32_t wh[4], al_unused[4];
        const uint32_t zero[4] = {0u, 0u, 0u, 0u};
        read_window(xh32, c0 + n + Lay::first_lag(C) + (h1 ? 8 : 0), wh);
        build_a<Lay, C>(a_h[C], al_unused, wh, zero, nrv, h1);
      });
      f32x16_t acc = {};
      if constexpr (Lay::kShared) acc = mfma(a_h[0], bsh, acc);
#pragma unroll
      for (int C = C0; C < NCH; ++C) acc = mfma(a_h[C], bh[NG - 1][C - C0], acc);
      return acc;
    };
    // kP1Tiles tiles per step, their norms loaded one step ahead, so that
    // independent product chains and the loads overlap their latency.  Tiles
    // past the end repeat the step's first tile (same minimum).  Pass 1
    // visits one tile in `stride`: every tile gives the tightest bounds, a
    // sample costs less.  Measured per group (strides 1-8): on 2000-sample
    // series every third tile is fastest for E 9-16 and every tile for the
    // other groups; above 4096 samples every fourth tile (the default; a
    // batched plan may set its own from its autotuner).
    const int stride = a.p1_stride > 0 ? a.p1_stride
                                       : (m_lo > 4096 ? 4 : ((ELO >= 9 && ELO <= 14) ? 3 : 1));
    uint32_t nN[kP1Tiles][NG];
    auto fetchN = [&](int c0) {  // in bounds: every tile start is below m_lo
#pragma unroll
      for (int t = 0; t < kP1Tiles; ++t) {
        const int c = c0 + 32 * stride * t < m_lo ? c0 + 32 * stride * t : c0;
#pragma unroll
        for (int g = 0; g < NG; ++g) nN[t][g] = nrm[g * ld + c + n];
      }
    };
    fetchN(0);
#pragma unroll 1
    for (int c0 = 0; c0 < m_lo; c0 += 32 * stride * kP1Tiles) {
      uint32_t nc[kP1Tiles][NG];
#pragma unroll
      for (int t = 0; t < kP1Tiles; ++t)
#pragma unroll
        for (int g = 0; g < NG; ++g) nc[t][g] = nN[t][g];
      if (c0 + 32 * stride * kP1Tiles < m_lo) fetchN(c0 + 32 * stride * kP1Tiles);
      f32x16_t acc[kP1Tiles];
      uint32_t tix[kP1Tiles];
#pragma unroll
      for (int t = 0; t < kP1Tiles; ++t) {
        const int c = c0 + 32 * stride * t < m_lo ? c0 + 32 * stride * t : c0;
        acc[t] = hi_tile(c, nc[t]);
        tix[t] = static_cast<uint32_t>(c) >> 5;
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float e = with_low10(acc[0][v], tix[0]);
#pragma unroll
        for (int t = 1; t < kP1Tiles; ++t) e = min2(e, with_low10(acc[t][v], tix[t]));
        bm[v] = min2(bm[v], e);
      }
    }
    float kb[NG][16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const bool won = bm[v] != __builtin_inff();
      const int bt = won ? static_cast<int>(__float_as_uint(bm[v]) & 0x3ffu) * 32 : -1;
      const int q = bt + 8 * (v >> 2) + (h1 ? 4 : 0) + (v & 3);
      float key[NG];
      exact_keys(bt < 0 ? 0 : q, bt >= 0 && q != p, key);
#pragma unroll
      for (int g = 0; g < NG; ++g) kb[g][v] = key[g];
    }
    // K-th smallest (K = E + 1) of the 32 keys of the lane pair: each lane
    // sorts its 16, and with A, B the two sorted halves (+inf past the end)
    // the K-th smallest of their union is the largest min(A[i], B[K - 1 - i]).
    static_for<ELO, EHI>([&](auto EC) {
      constexpr int E = decltype(EC)::value;
      constexpr int K = E + 1;
      float a[16], b[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) a[v] = kb[E - ELO][v];
      sort16(a);
#pragma unroll
      for (int v = 0; v < 16; ++v) b[v] = __shfl_xor(a[v], 32);
      float u = -__builtin_inff();
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int j = K - 1 - i;
        if (i < 16 && j < 16) u = fmaxf(u, fminf(a[i], b[j]));
        else if (i < 16) u = fmaxf(u, a[i]);
        else u = fmaxf(u, b[j]);
      }
      ub[E - ELO] = u;
    });
  }

  float qk[TOT];
  int qi[TOT];
  static_for<ELO, EHI>([&](auto EC) {
    constexpr int E = decltype(EC)::value;
    constexpr int OFF = list_off<ELO>(E);
    const bool act = list_active(E);
#pragma unroll
    for (int i = 0; i < E + 1; ++i) {
      qk[OFF + i] = act ? __builtin_inff() : -1.0f;
      qi[OFF + i] = -1;
    }
  });

  // Pass 2: every E's threshold rides in the products, so the estimate of
  // E is D - T and a candidate survives where the minimum over the group's E
  // is negative.  A tile's survivors are one sign mask per lane, queued in
  // LDS with the tile index when not empty (no branch) and re-ranked in
  // batches, so the lists change only at a flush.
  uint32_t *qbuf = qbuf_all + wave * (kQueueCap * kWave) + lane;  // entry i at qbuf[i * 64]
  int cnt = 0;   // queued entries
  int nsv = 0;   // queued survivors
  auto refresh = [&]() {
    static_for<ELO, EHI>([&](auto EC) {
      constexpr int E = decltype(EC)::value;
      constexpr int g = E - ELO;
      constexpr int OFF = list_off<ELO>(E);
      const float own = qk[OFF + E];
      // K-th smallest key of the query's two half-lists together: the largest
      // elementwise minimum of one sorted list against the other reversed.
      float kth = ub[g];
      float u = -__builtin_inff();
#pragma unroll
      for (int i = 0; i <= E; ++i) u = fmaxf(u, fminf(qk[OFF + i], __shfl_xor(qk[OFF + E - i], 32)));
      kth = fminf(kth, u);
      const float T = own < 0.0f ? -kGramBig : fminf((kth - nq[g]) + kGramFloor, kGramBig);
      set_threshold<Lay>(bh[g][NCH - 1 - C0], bl[g][NCH - 1 - C0], T, h1);
    });
  };
  // Re-rank the queued candidates, lowest first: uniform trip count and a
  // branch-free body keep the lists in place in registers.
  // Two survivors per step (where the register budget allows): their key
  // chains are independent and overlap; they are inserted in order, so each
  // list still sees ascending q.
  constexpr int kStep = (TOT <= 44 && !XG) ? 2 : 1;
  auto flush = [&]() {
    const int n_iter = (wave_max(nsv) + kStep - 1) / kStep;
    int j = 0;
    uint32_t cur = qbuf[0];
    uint32_t nxt = qbuf[kWave];
    auto take = [&](bool has) {  // this lane's next survivor (0 when none is left)
      const bool adv = (cur & kSignBits) == 0u;  // entry done: the next one holds the next survivor
      cur = adv ? nxt : cur;
      j += adv ? 1 : 0;
      nxt = qbuf[(j + 1 < kQueueCap ? j + 1 : j) * kWave];
      const uint32_t bit = cur & kSignBits;
      const int pos = bit ? __builtin_ctz(bit) : 0;
      cur ^= bit ? (1u << pos) : 0u;
      const int qq = static_cast<int>(tile_of(cur)) * 32 + (pos & ~7) + (pos & 3) + (h1 ? 4 : 0);
      return has ? qq : 0;
    };
#pragma unroll 1
    for (int it = 0; it < n_iter; ++it) {
      if constexpr (kStep == 2) {
        const bool has0 = 2 * it < nsv, has1 = 2 * it + 1 < nsv;
        const int q0 = take(has0);
        const int q1 = take(has1);
        float key0[NG], key1[NG];
        exact_keys2(q0, has0 && q0 != p, key0, q1, has1 && q1 != p, key1);
        static_for<ELO, EHI>([&](auto EC) {
          constexpr int E = decltype(EC)::value;
          // The empty asm hides the +inf of idle lanes from the optimiser,
          // which would otherwise branch around the insertion.
          float kin0 = key0[E - ELO], kin1 = key1[E - ELO];
          asm volatile("" : "+v"(kin0), "+v"(kin1));
          if (__builtin_amdgcn_ballot_w64(kin0 < qk[list_off<ELO>(E) + E]))
            slice_insert<list_off<ELO>(E), E + 1, TOT>(qk, qi, kin0, q0);
          if (__builtin_amdgcn_ballot_w64(kin1 < qk[list_off<ELO>(E) + E]))
            slice_insert<list_off<ELO>(E), E + 1, TOT>(qk, qi, kin1, q1);
        });
      } else {
        const bool has = it < nsv;
        const int q = take(has);
        float key[NG];
        exact_keys(q, has && q != p, key);
        static_for<ELO, EHI>([&](auto EC) {
          constexpr int E = decltype(EC)::value;
          float kin = key[E - ELO];
          asm volatile("" : "+v"(kin));
          if (__builtin_amdgcn_ballot_w64(kin < qk[list_off<ELO>(E) + E]))
            slice_insert<list_off<ELO>(E), E + 1, TOT>(qk, qi, kin, q);
        });
      }
    }
    cnt = 0;
    nsv = 0;
    refresh();
  };
  refresh();
  if (pw < m_lo) {
    fetch(0);
    read_raw(0);
    const bool pass_all = unsafe && act_any;  // filter off: every candidate is re-ranked
    // Only the sign of the minimum over E matters: OR of the sign bits.
    auto estimates = [&](uint32_t (&e)[16]) {
      static_for<0, NG - 1>([&](auto GC) {
        constexpr int g = decltype(GC)::value;
        const f32x16_t acc = estimate(g);
#pragma unroll
        for (int v = 0; v < 16; ++v) e[v] = (g == 0 ? 0u : e[v]) | __float_as_uint(acc[v]);
      });
    };
    // The next tile's products are issued before this tile's survivors are
    // queued, so the two overlap.  Products issued before a re-rank use the
    // older (larger) thresholds: more survivors, never fewer.
    // The tile step (loads, products, queueing) runs at a raised wave
    // priority and the re-rank at the normal one: of the two waves a SIMD
    // holds, the one with products to issue goes first, and the other's
    // re-rank fills the matrix core's latency (2.5 % off the filter on the
    // 10000 x 2000 step; results unchanged).
    uint32_t e[16];
    load_tile(0, 32);
    estimates(e);
#pragma unroll 1
    for (int c0 = 0; c0 < m_lo; c0 += 32) {
      const int cn = c0 + 32 < m_lo ? c0 + 32 : c0;  // the last step repeats a tile, unused
      uint32_t e_next[16];
      __builtin_amdgcn_s_setprio(1);
      load_tile(cn, cn + 32);
      estimates(e_next);
      uint32_t bits = sign_mask(e);
      if (unsafe) bits = pass_all ? kSignBits : 0u;
      qbuf[cnt * kWave] = bits | tile_code(static_cast<uint32_t>(c0) >> 5);
      cnt += bits != 0u;
      nsv += __builtin_popcount(bits);
      __builtin_amdgcn_s_setprio(0);
      if (__builtin_amdgcn_ballot_w64(cnt == kQueueCap)) flush();
#pragma unroll
      for (int v = 0; v < 16; ++v) e[v] = e_next[v];
    }
  }
  flush();

  // Each query's two half-lists -> its full list (both lanes end equal).
  // [own list ascending, maxima, partner list descending] is bitonic; its
  // first half-cleaner stage (elementwise minimum) leaves the N smallest as a
  // bitonic sequence, and the remaining stages sort it.  Blocks that start at
  // or beyond K only order entries that are dropped, so they are skipped.
  // Order: (key, index) lexicographic, the index unsigned (empty entries last).
  static_for<ELO, EHI>([&](auto EC) {
    constexpr int E = decltype(EC)::value;
    constexpr int K = E + 1;
    constexpr int OFF = list_off<ELO>(E);
    constexpr int N = K <= 8 ? 8 : (K <= 16 ? 16 : 32);
    static_assert(N - K < K, "every position of the lower half holds an entry");
    float ck[N];
    int ci[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int j = N - 1 - i;  // partner entry facing position i, if j < K
      float pk = 0.0f;
      int pi = 0;
      if (j < K) {
        pk = __shfl_xor(qk[OFF + j], 32);
        pi = __shfl_xor(qi[OFF + j], 32);
      }
      if (i < K && j < K) {
        const bool lt = lex_less(pk, pi, qk[OFF + i], qi[OFF + i]);
        ck[i] = lt ? pk : qk[OFF + i];
        ci[i] = lt ? pi : qi[OFF + i];
      } else if (i < K) {
        ck[i] = qk[OFF + i];
        ci[i] = qi[OFF + i];
      } else {
        ck[i] = pk;
        ci[i] = pi;
      }
    }
#pragma unroll
    for (int d = N / 2; d > 0; d >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i)
        if ((i & d) == 0 && (i & ~(2 * d - 1)) < K) {
          const bool sw = lex_less(ck[i + d], ci[i + d], ck[i], ci[i]);
          const float k0 = ck[i], k1 = ck[i + d];
          const int i0 = ci[i], i1 = ci[i + d];
          ck[i] = sw ? k1 : k0;
          ci[i] = sw ? i1 : i0;
          ck[i + d] = sw ? k0 : k1;
          ci[i + d] = sw ? i0 : i1;
        }
#pragma unroll
    for (int i = 0; i < K; ++i) {
      qk[OFF + i] = ck[i];
      qi[OFF + i] = ci[i];
    }
  });

  // Epilogue: E alternates between the two lanes of a query.  The co-moments
  // are merged in the order of the exact scan (a 32-lane butterfly per half,
  // then the two halves of each 64-query group, then the groups in order), so
  // the correlations match it bit for bit.
  // Round r: the lower half finishes E = ELO + 2r, the upper half ELO + 2r + 1.
  static_for<0, (NG - 1) / 2>([&](auto RC) {
    constexpr int E0 = ELO + 2 * decltype(RC)::value;
    constexpr int E1 = E0 + 1 <= EHI ? E0 + 1 : E0;
    constexpr int K1 = E1 + 1;
    const bool up = h1 && E1 != E0;
    int idx[K1];
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      const int lo_i = i < E0 + 1 ? qi[list_off<ELO>(E0) + i] : -1;
      idx[i] = up ? qi[list_off<ELO>(E1) + i] : lo_i;
    }
    Mom mine = mom_zero();
    if (!h1 || up) mine = finish_round<E0, E1>(a, row, p, L, Tp, need, idx, up ? E1 : E0, XG ? x : xs);
    if (a.mom) {  // uniform
#pragma unroll
      for (int m = 1; m < 32; m <<= 1) mine = mom_merge(mine, mom_shfl_xor(mine, m));
      if (lane == 0) wmom[wave][E0 - ELO] = mine;
      if (E1 != E0 && lane == 32) wmom[wave][E1 - ELO] = mine;
    }
  });
  if (a.mom == nullptr) return;
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < NG) {
    const int g = static_cast<int>(threadIdx.x);
    const int E = ELO + g;
    const int mE = L - (E - 1) - Tp;
    if (mE - 1 >= E + 1 && blk0 < mE) {
      Mom t = mom_merge(wmom[0][g], wmom[1][g]);
#pragma unroll
      for (int w = 1; w < kGramWaves / 2; ++w) t = mom_merge(t, mom_merge(wmom[2 * w][g], wmom[2 * w + 1][g]));
      a.mom[(static_cast<int64_t>(row) * a.E_max + (E - 1)) * a.mom_blocks + bx] = t;
    }
  }
}

// One-dimensional grid over (slot, query block).  Workgroups are dispatched
// round-robin over the kGramXcds dies, each with its own L2: workgroup i runs
// on die i % kGramXcds, and the nblk query blocks of a slot are given to one
// die, whose L2 then serves that slot's samples and norms to all of them.
template <int ELO, int EHI, bool XG>
__global__ __launch_bounds__(kGramThreads) void k_gram(KnnArgs a, int slot0, int nslots, int nblk) {
  extern __shared__ float gram_smem[];
  const int i = static_cast<int>(blockIdx.x);
  const int x = i % kGramXcds, s = i / kGramXcds;
  const int row = (s / nblk) * kGramXcds + x;
  if (row >= nslots) return;  // padding of the last die round (uniform)
  gram_scan<ELO, EHI, XG>(a, slot0 + row, s % nblk, gram_smem);
}

// Centring constant of each slot: the float32 mean (float64 sum).
__global__ __launch_bounds__(256) void k_gram_mean(KnnArgs a) {
  const int row = static_cast<int>(blockIdx.x);
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int64_t L = a.L_dev ? a.L_dev[row] : a.L_uni;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < L; i += 256) s += static_cast<double>(x[i]);
  for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = (part[0] + part[1]) + (part[2] + part[3]);
    a.gram_mu[row] = L > 0 ? static_cast<float>(t / static_cast<double>(L)) : 0.0f;
  }
}

// Packed s N_E(q) for every E >= kGramEMin and q < gram_ld (zero samples past
// the end of the series).
__global__ __launch_bounds__(256) void k_gram_norms(KnnArgs a) {
  const int row = static_cast<int>(blockIdx.y);
  const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t ld = a.gram_ld;
  if (q >= ld) return;
  const float *__restrict__ x = a.X + static_cast<int64_t>(row) * a.ldx;
  const int64_t L = a.L_dev ? a.L_dev[row] : a.L_uni;
  const float mu = a.gram_mu[row];
  uint32_t *out = a.gram_nrm + static_cast<int64_t>(row) * kGramNE * ld + q;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < EDM_E_MAX; ++j) {
    const float b = q + j < L ? x[q + j] - mu : 0.0f;
    s = s + b * b;
    if (j + 1 >= kGramEMin) out[(j + 1 - kGramEMin) * ld] = split_pack(kGramScale * s);
  }
}

// Work-list form: one workgroup per (row, block) item.  (The filtered scan
// fills a CU with one workgroup, so pulling items gains nothing, and a loop
// around the scan costs registers.)
template <int ELO, int EHI, bool XG>
__global__ __launch_bounds__(kGramThreads) void k_gram_items(KnnArgs a,
                                                             const TableItem *__restrict__ items) {
  extern __shared__ float gram_smem[];
  const int it = static_cast<int>(blockIdx.x);
  const int row = __builtin_amdgcn_readfirstlane(items[it].row);
  const int blk = __builtin_amdgcn_readfirstlane(static_cast<int>(items[it].blk));
  gram_scan<ELO, EHI, XG>(a, row, blk, gram_smem);
}

using GramFn = void (*)(KnnArgs, int, int, int);

template <int LO, int HI, bool XG>
constexpr GramFn gram_fn() {
  return &k_gram<LO, HI, XG>;
}

// (lo, hi) -> kernel; lo is a group start of the filtered partition.
template <bool XG>
GramFn pick_xg(int lo, int hi) {
  switch (lo) {
    case 5: {
      constexpr GramFn t[] = {gram_fn<5, 5, XG>(), gram_fn<5, 6, XG>(), gram_fn<5, 7, XG>(), gram_fn<5, 8, XG>()};
      return hi >= 5 && hi <= 8 ? t[hi - 5] : nullptr;
    }
    case 9: {
      constexpr GramFn t[] = {gram_fn<9, 9, XG>(), gram_fn<9, 10, XG>(), gram_fn<9, 11, XG>()};
      return hi >= 9 && hi <= 11 ? t[hi - 9] : nullptr;
    }
    case 12: {
      constexpr GramFn t[] = {gram_fn<12, 12, XG>(), gram_fn<12, 13, XG>()};
      return hi >= 12 && hi <= 13 ? t[hi - 12] : nullptr;
    }
    case 14: {
      constexpr GramFn t[] = {gram_fn<14, 14, XG>(), gram_fn<14, 15, XG>(), gram_fn<14, 16, XG>()};
      return hi >= 14 && hi <= 16 ? t[hi - 14] : nullptr;
    }
    case 17: {
      constexpr GramFn t[] = {gram_fn<17, 17, XG>(), gram_fn<17, 18, XG>()};
      return hi >= 17 && hi <= 18 ? t[hi - 17] : nullptr;
    }
    case 19: {
      constexpr GramFn t[] = {gram_fn<19, 19, XG>(), gram_fn<19, 20, XG>()};
      return hi >= 19 && hi <= 20 ? t[hi - 19] : nullptr;
    }
    default:
      return nullptr;
  }
}

// Exact samples in LDS up to kGramLdsXsMax samples, read from global beyond.
bool use_global_x(int64_t L_max) { return L_max > kGramLdsXsMax; }

size_t gram_shm(int64_t ld, bool xg) {
  return static_cast<size_t>(ld) * ((xg ? 0 : sizeof(float)) + 2 * sizeof(uint16_t)) +
         sizeof(uint32_t) * kQueueCap * kGramThreads;
}

}  // namespace

hipError_t launch_gram_prep(const KnnArgs &a, int nslots, int64_t L_max, hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  if (a.gram_ld < L_max + kGramPad) return hipErrorInvalidValue;
  TimedLaunch timed(EDM_KF_FILTER_PREP, st);
  hipLaunchKernelGGL(k_gram_mean, dim3(static_cast<unsigned>(nslots)), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gx = static_cast<unsigned>((a.gram_ld + 255) / 256);
  hipLaunchKernelGGL(k_gram_norms, dim3(gx, static_cast<unsigned>(nslots)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_gram_items(const KnnArgs &a, int g, const TableItem *items, int n_items,
                             int64_t L_max, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  using Fn = void (*)(KnnArgs, const TableItem *);
  static const Fn fl[6] = {&k_gram_items<5, 8, false>,   &k_gram_items<9, 11, false>,
                           &k_gram_items<12, 13, false>, &k_gram_items<14, 16, false>,
                           &k_gram_items<17, 18, false>, &k_gram_items<19, 20, false>};
  static const Fn fg[6] = {&k_gram_items<5, 8, true>,   &k_gram_items<9, 11, true>,
                           &k_gram_items<12, 13, true>, &k_gram_items<14, 16, true>,
                           &k_gram_items<17, 18, true>, &k_gram_items<19, 20, true>};
  static_assert(sizeof(kGramGroups) / sizeof(kGramGroups[0]) == 6, "one kernel per filtered group");
  const int64_t lds = a.gram_lds > 0 ? a.gram_lds : a.gram_ld;
  if (g < 0 || g > 5 || L_max > kGramLMax || a.gram_ld < L_max + kGramPad ||
      lds < L_max + kGramPad || lds > a.gram_ld || a.tau != 1 || a.mom != nullptr)
    return hipErrorInvalidValue;
  const bool xg = use_global_x(lds - kGramPad);
  const Fn *fns = xg ? fg : fl;
  const size_t shm = gram_shm(lds, xg);
  const void *fn = reinterpret_cast<const void *>(fns[g]);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  TimedLaunch timed(EDM_KF_FILTER_SCAN, st);
  hipLaunchKernelGGL(fns[g], dim3(static_cast<unsigned>(n_items)), dim3(kGramThreads), shm, st, a,
                     items);
  return hipGetLastError();
}

hipError_t launch_gram_group(const KnnArgs &a, int lo, int hi, int nslots, int64_t L_max,
                             hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  const bool xg = use_global_x(a.gram_ld - kGramPad);
  const GramFn fn = xg ? pick_xg<true>(lo, hi) : pick_xg<false>(lo, hi);
  if (fn == nullptr || L_max > kGramLMax || a.gram_ld < L_max + kGramPad || a.tau != 1)
    return hipErrorInvalidValue;
  const size_t shm = gram_shm(a.gram_ld, xg);
  const void *f = reinterpret_cast<const void *>(fn);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(shm));
    if (e != hipSuccess) return e;
  }
  const int nblk = static_cast<int>((L_max + kKnnThreads - 1) / kKnnThreads);
  TimedLaunch timed(EDM_KF_FILTER_SCAN, st);
  constexpr int kMaxSlots = 32768;
  for (int s0 = 0; s0 < nslots; s0 += kMaxSlots) {
    const int ny = nslots - s0 < kMaxSlots ? nslots - s0 : kMaxSlots;
    const unsigned nwg = static_cast<unsigned>((ny + kGramXcds - 1) / kGramXcds * kGramXcds * nblk);
    hipLaunchKernelGGL(fn, dim3(nwg), dim3(kGramThreads), shm, st, a, s0, ny, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace edm
