// Device-side helpers shared by the libedm kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace edm {

constexpr int kWave = 64;

// Co-moments of a set of (observation, prediction) pairs: count, means and
// centred second moments.  Two sets merge exactly with the pairwise update of
// Chan, Golub & LeVeque, which is the stable covariance form the paper uses
// for its on-the-fly Pearson reduction (Section 3.4, after Schubert & Gertz).
struct Mom {
  double n, mo, mp, coo, cpp, cop;
};

__device__ __forceinline__ Mom mom_zero() { return Mom{0.0, 0.0, 0.0, 0.0, 0.0, 0.0}; }

__device__ __forceinline__ Mom mom_merge(const Mom &a, const Mom &b) {
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  const double n = a.n + b.n;
  const double fb = b.n / n;
  const double f = a.n * fb;
  const double dO = b.mo - a.mo;
  const double dP = b.mp - a.mp;
  Mom r;
  r.n = n;
  r.mo = a.mo + dO * fb;
  r.mp = a.mp + dP * fb;
  r.coo = a.coo + b.coo + dO * dO * f;
  r.cpp = a.cpp + b.cpp + dP * dP * f;
  r.cop = a.cop + b.cop + dO * dP * f;
  return r;
}

// Moments of c points summarised by raw sums of values shifted by reference
// values taken from the points themselves (so = sum(o - ref_o),
// soo = sum((o - ref_o)^2), ...).  The shift keeps the raw sums free of
// cancellation for data of any offset, and a constant series gives exactly
// zero spread.
__device__ __forceinline__ Mom mom_from_shifted_sums(double c, double ref_o, double ref_p,
                                                     double so, double sp, double soo,
                                                     double spp, double sop) {
  if (c == 0.0) return mom_zero();
  const double ao = so / c, ap = sp / c;
  Mom r;
  r.n = c;
  r.mo = ref_o + ao;
  r.mp = ref_p + ap;
  r.coo = fmax(soo - so * ao, 0.0);
  r.cpp = fmax(spp - sp * ap, 0.0);
  r.cop = sop - so * ap;
  return r;
}

__device__ __forceinline__ Mom mom_shfl_xor(const Mom &a, int m) {
  Mom r;
  r.n = __shfl_xor(a.n, m);
  r.mo = __shfl_xor(a.mo, m);
  r.mp = __shfl_xor(a.mp, m);
  r.coo = __shfl_xor(a.coo, m);
  r.cpp = __shfl_xor(a.cpp, m);
  r.cop = __shfl_xor(a.cop, m);
  return r;
}

// Butterfly merge across the 64 lanes of a wave; every lane ends with the total.
__device__ __forceinline__ Mom mom_wave_reduce(Mom a) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) a = mom_merge(a, mom_shfl_xor(a, m));
  return a;
}

// Pearson correlation from merged co-moments; NaN when either side has no
// spread (Section 2.1 step 4).
__device__ __forceinline__ double mom_rho(const Mom &a) {
  if (!(a.coo > 0.0) || !(a.cpp > 0.0)) return __builtin_nan("");
  return a.cop / sqrt(a.coo * a.cpp);
}

}  // namespace edm
